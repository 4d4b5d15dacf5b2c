// C ABI of the surrogate network: forward, training step (forward, MSE, backward, Adam), BF16
// weight refresh, surrogate likelihood and a general BF16 product.  Arithmetic runs in k_mlp.hip.
#include <algorithm>
#include <hip/hip_runtime.h>
#include <math.h>

#include <vector>

#include "pcmd_ctx.h"
#include "pcmd_mlp.h"

using namespace pcmd;

namespace {

constexpr int MLP_LOSS_CHUNK = 1024;  // rows per forward pass of pcmd_mlp_loss

struct Layout {
  int L = 0;
  int d[PCMD_MLP_MAX_LAYERS + 1] = {};
  int64_t off[PCMD_MLP_MAX_LAYERS + 1] = {};   // master offset of W_l (b_l follows)
  int64_t woff[PCMD_MLP_MAX_LAYERS + 1] = {};  // bf16 offset of W_l
  int dmax = 0;
  int64_t params = 0, weights = 0, flops_per_sample = 0;
};

bool make_layout(const int32_t *dims, int32_t n_layers, Layout &lay) {
  if (!dims || n_layers < 1 || n_layers > PCMD_MLP_MAX_LAYERS) return false;
  lay.L = n_layers;
  int64_t o = 0, w = 0;
  for (int l = 0; l <= n_layers; ++l) {
    if (dims[l] < 1 || dims[l] > 65536) return false;
    lay.d[l] = dims[l];
    if (dims[l] > lay.dmax) lay.dmax = dims[l];
  }
  for (int l = 0; l < n_layers; ++l) {
    lay.off[l] = o;
    lay.woff[l] = w;
    o += (int64_t)dims[l + 1] * dims[l] + dims[l + 1];
    w += (int64_t)dims[l + 1] * dims[l];
    lay.flops_per_sample += 2 * (int64_t)dims[l + 1] * dims[l];
  }
  lay.params = o;
  lay.weights = w;
  return true;
}

int check_net(pcmd_ctx *c, const pcmd_mlp *net, Layout &lay, const char *who) {
  if (!net) return fail(c, PCMD_E_INVAL, "%s: null network", who);
  if (!make_layout(net->dims, net->n_layers, lay)) return fail(c, PCMD_E_INVAL, "%s: bad layer sizes", who);
  if (!net->master || !net->w_bf16 || !net->wt_bf16) return fail(c, PCMD_E_INVAL, "%s: null weights", who);
  return PCMD_OK;
}

// forward through all layers; activations kept in the context for a following backward pass.
// Sample k of the batch reads input row rows[k] of x (row k when rows is NULL).
hipError_t forward_impl(pcmd_ctx *c, const pcmd_mlp *net, const Layout &lay, int n, const float *x,
                        const int32_t *rows, int64_t n_total, float *y_out, hipStream_t s) {
  __bf16 *act = (__bf16 *)c->mlp_act.p;
  float *pre = (float *)c->mlp_pre.p;
  const __bf16 *w = (const __bf16 *)net->w_bf16;
  hipError_t e = rows ? launch_gather_f32_to_bf16(x, rows, n_total, lay.d[0], n, act, c->status, s)
                      : launch_f32_to_bf16(x, act, (int64_t)n * lay.d[0], s);
  int64_t aoff = 0, poff = 0;
  for (int l = 0; l < lay.L && e == hipSuccess; ++l) {
    const int din = lay.d[l], dout = lay.d[l + 1];
    GemmArgs g{};
    g.M = n;
    g.N = dout;
    g.K = din;
    g.A = act + aoff;
    g.lda = din;
    g.B = w + lay.woff[l];
    g.ldb = din;
    g.bias = net->master + lay.off[l] + (int64_t)dout * din;
    g.ldc = dout;
    const bool last = l == lay.L - 1;
    g.C = (last && y_out) ? y_out : pre + poff;
    if (!last) {
      g.Cb = act + aoff + (int64_t)n * din;
      g.ldcb = dout;
    }
    {
      ScopedTimer tm(c, PCMD_TIMER_GEMM, 2.0 * (double)n * (double)din * (double)dout, s);
      e = launch_gemm(g, false, false, last ? EPI_BIAS : EPI_BIAS_GELU, c->mlp_ws.p, c->mlp_ws.n, s);
    }
    aoff += (int64_t)n * din;
    poff += (int64_t)n * dout;
  }
  return e;
}

int ensure_mlp_scratch(pcmd_ctx *c, const Layout &lay, int n) {
  int64_t acts = 0, pres = 0;
  for (int l = 0; l < lay.L; ++l) {
    acts += (int64_t)n * lay.d[l];
    pres += (int64_t)n * lay.d[l + 1];
  }
  int r;
  if ((r = ensure(c, c->mlp_act, (size_t)(acts + (int64_t)n * lay.dmax) * 2, "network activations"))) return r;
  if ((r = ensure(c, c->mlp_pre, (size_t)pres * 4, "network pre-activations"))) return r;
  if ((r = ensure(c, c->mlp_dza, (size_t)n * lay.dmax * 2, "network gradients"))) return r;
  if ((r = ensure(c, c->mlp_dzb, (size_t)n * lay.dmax * 2, "network gradients"))) return r;
  if ((r = ensure(c, c->mlp_grad, (size_t)lay.params * 4, "parameter gradients"))) return r;
  if ((r = ensure(c, c->mlp_part, 256 * 8, "loss partials"))) return r;
  // GEMM workspace: the largest over the forward, weight-gradient and input-gradient products
  size_t ws = 0;
  for (int l = 0; l < lay.L; ++l) {
    const int din = lay.d[l], dout = lay.d[l + 1];
    ws = std::max(ws, gemm_workspace_bytes(n, dout, din, false, false));
    ws = std::max(ws, gemm_workspace_bytes(dout, din, n, true, true));
    ws = std::max(ws, gemm_workspace_bytes(n, din, dout, false, false));
  }
  if (ws && (r = ensure(c, c->mlp_ws, ws, "GEMM workspace"))) return r;
  return PCMD_OK;
}

// Forward, mean squared error and backward of one batch into grad (FP32, packed like the
// master parameters).  Targets of sample k are row rows[k] of t (row k when rows is NULL).
hipError_t backward_impl(pcmd_ctx *c, const pcmd_mlp *net, const Layout &lay, int n, const float *x, const float *t,
                         const int32_t *rows, int64_t n_total, float *loss_out, float *grad, hipStream_t s) {
  hipError_t e = forward_impl(c, net, lay, n, x, rows, n_total, nullptr, s);
  std::vector<int64_t> aoffs(lay.L), poffs(lay.L);
  {
    int64_t ao = 0, po = 0;
    for (int l = 0; l < lay.L; ++l) {
      aoffs[l] = ao;
      poffs[l] = po;
      ao += (int64_t)n * lay.d[l];
      po += (int64_t)n * lay.d[l + 1];
    }
  }
  __bf16 *act = (__bf16 *)c->mlp_act.p;
  float *pre = (float *)c->mlp_pre.p;
  __bf16 *dz = (__bf16 *)c->mlp_dza.p, *dz2 = (__bf16 *)c->mlp_dzb.p;
  const int dL = lay.d[lay.L];
  const double scale = 1.0 / ((double)n * (double)dL);
  // output layer pre-activations are the prediction
  if (e == hipSuccess)
    e = launch_mse_grad(pre + poffs[lay.L - 1], t, (int64_t)n * dL, dL, rows, n_total, scale, dz,
                        (double *)c->mlp_part.p, loss_out, c->status, s);
  for (int l = lay.L - 1; l >= 0 && e == hipSuccess; --l) {
    const int din = lay.d[l], dout = lay.d[l + 1];
    GemmArgs gw{};
    gw.M = dout;
    gw.N = din;
    gw.K = n;
    gw.A = dz;
    gw.lda = dout;
    gw.B = act + aoffs[l];
    gw.ldb = din;
    gw.C = grad + lay.off[l];
    gw.ldc = din;
    {
      ScopedTimer tm(c, PCMD_TIMER_GEMM, 2.0 * (double)n * (double)din * (double)dout, s);
      e = launch_gemm(gw, true, true, EPI_STORE, c->mlp_ws.p, c->mlp_ws.n, s);
    }
    if (e == hipSuccess) e = launch_colsum(dz, n, dout, grad + lay.off[l] + (int64_t)dout * din, s);
    if (e == hipSuccess && l > 0) {
      GemmArgs gx{};
      gx.M = n;
      gx.N = din;
      gx.K = dout;
      gx.A = dz;
      gx.lda = dout;
      gx.B = (const __bf16 *)net->wt_bf16 + lay.woff[l];
      gx.ldb = dout;
      gx.Cb = dz2;
      gx.ldcb = din;
      gx.Z = pre + poffs[l - 1];
      gx.ldz = din;
      {
        ScopedTimer tm(c, PCMD_TIMER_GEMM, 2.0 * (double)n * (double)din * (double)dout, s);
        e = launch_gemm(gx, false, false, EPI_GELU_GRAD, c->mlp_ws.p, c->mlp_ws.n, s);
      }
      __bf16 *tmp = dz;
      dz = dz2;
      dz2 = tmp;
    }
  }
  return e;
}

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected for step `step`) per layer,
// refreshing the BF16 copies of W and W^T.
hipError_t adam_impl(const pcmd_mlp *net, const Layout &lay, const float *grad, float lr, int step, hipStream_t s) {
  const double bc1 = 1.0 - pow(0.9, (double)step), bc2 = 1.0 - pow(0.999, (double)step);
  hipError_t e = hipSuccess;
  for (int l = 0; l < lay.L && e == hipSuccess; ++l) {
    AdamArgs a{};
    a.n_out = lay.d[l + 1];
    a.n_in = lay.d[l];
    a.update = 1;
    a.master = net->master + lay.off[l];
    a.m = net->adam_m + lay.off[l];
    a.v = net->adam_v + lay.off[l];
    a.grad = grad + lay.off[l];
    a.w_bf16 = net->w_bf16 + lay.woff[l];
    a.wt_bf16 = net->wt_bf16 + lay.woff[l];
    a.lr = lr;
    a.beta1 = 0.9f;
    a.beta2 = 0.999f;
    a.eps = 1e-8f;
    a.bc1 = (float)bc1;
    a.bc2 = (float)bc2;
    e = launch_adam_layer(a, s);
  }
  return e;
}

}  // namespace

extern "C" {

int64_t pcmd_mlp_param_count(const int32_t *dims, int32_t n_layers) {
  Layout lay;
  return make_layout(dims, n_layers, lay) ? lay.params : -1;
}

int64_t pcmd_mlp_weight_count(const int32_t *dims, int32_t n_layers) {
  Layout lay;
  return make_layout(dims, n_layers, lay) ? lay.weights : -1;
}

int pcmd_mlp_refresh(pcmd_ctx *c, const pcmd_mlp *net, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  Layout lay;
  int r = check_net(c, net, lay, "pcmd_mlp_refresh");
  if (r) return r;
  DeviceGuard dg(c->device);
  for (int l = 0; l < lay.L; ++l) {
    AdamArgs a{};
    a.n_out = lay.d[l + 1];
    a.n_in = lay.d[l];
    a.update = 0;
    a.master = net->master + lay.off[l];
    a.w_bf16 = net->w_bf16 + lay.woff[l];
    a.wt_bf16 = net->wt_bf16 + lay.woff[l];
    hipError_t e = launch_adam_layer(a, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "pcmd_mlp_refresh");
  }
  c->err.clear();
  return PCMD_OK;
}

int pcmd_mlp_forward(pcmd_ctx *c, const pcmd_mlp *net, int32_t n, const float *x, float *y, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  Layout lay;
  int r = check_net(c, net, lay, "pcmd_mlp_forward");
  if (r) return r;
  if (n < 1 || !x || !y) return fail(c, PCMD_E_INVAL, "pcmd_mlp_forward: bad batch or null pointer");
  DeviceGuard dg(c->device);
  if ((r = ensure_mlp_scratch(c, lay, n))) return r;
  hipError_t e = forward_impl(c, net, lay, n, x, nullptr, n, y, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_mlp_forward");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_mlp_backward(pcmd_ctx *c, const pcmd_mlp *net, int32_t n, const float *x, const float *t,
                      const int32_t *rows, int64_t n_total, float *loss_out, float *grad_out, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  Layout lay;
  int r = check_net(c, net, lay, "pcmd_mlp_backward");
  if (r) return r;
  if (n < 1 || !x || !t || !grad_out) return fail(c, PCMD_E_INVAL, "pcmd_mlp_backward: bad batch or null pointer");
  if (rows && n_total < 1) return fail(c, PCMD_E_INVAL, "pcmd_mlp_backward: n_total must be >= 1 with a row vector");
  DeviceGuard dg(c->device);
  if ((r = ensure_mlp_scratch(c, lay, n))) return r;
  hipError_t e = backward_impl(c, net, lay, n, x, t, rows, n_total, loss_out, grad_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_mlp_backward");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_mlp_adam(pcmd_ctx *c, const pcmd_mlp *net, const float *grad, float lr, int32_t step, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  Layout lay;
  int r = check_net(c, net, lay, "pcmd_mlp_adam");
  if (r) return r;
  if (!grad || !net->adam_m || !net->adam_v || step < 1 || !(lr >= 0.0f) || !isfinite(lr))
    return fail(c, PCMD_E_INVAL, "pcmd_mlp_adam: needs a gradient, moments, step >= 1 and a finite lr >= 0");
  DeviceGuard dg(c->device);
  hipError_t e = adam_impl(net, lay, grad, lr, step, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_mlp_adam");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_mlp_train_step(pcmd_ctx *c, const pcmd_mlp *net, int32_t n, const float *x, const float *t, float lr,
                        int32_t step, float *loss_out, float *grad_out, int32_t apply_update, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  Layout lay;
  int r = check_net(c, net, lay, "pcmd_mlp_train_step");
  if (r) return r;
  if (n < 1 || !x || !t) return fail(c, PCMD_E_INVAL, "pcmd_mlp_train_step: bad batch or null pointer");
  if (apply_update && (!net->adam_m || !net->adam_v || step < 1 || !(lr >= 0.0f) || !isfinite(lr)))
    return fail(c, PCMD_E_INVAL, "pcmd_mlp_train_step: Adam needs moments, step >= 1 and a finite lr >= 0");
  DeviceGuard dg(c->device);
  if ((r = ensure_mlp_scratch(c, lay, n))) return r;
  hipStream_t s = (hipStream_t)stream;
  float *grad = grad_out ? grad_out : (float *)c->mlp_grad.p;
  hipError_t e = backward_impl(c, net, lay, n, x, t, nullptr, n, loss_out, grad, s);
  if (e == hipSuccess && apply_update) e = adam_impl(net, lay, grad, lr, step, s);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_mlp_train_step");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_mlp_loss(pcmd_ctx *c, const pcmd_mlp *net, int32_t n, const float *x, const float *t, const int32_t *rows,
                  int64_t n_total, double *mse_out, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  Layout lay;
  int r = check_net(c, net, lay, "pcmd_mlp_loss");
  if (r) return r;
  if (n < 1 || !x || !t || !mse_out) return fail(c, PCMD_E_INVAL, "pcmd_mlp_loss: bad set or null pointer");
  if (rows && n_total < 1) return fail(c, PCMD_E_INVAL, "pcmd_mlp_loss: n_total must be >= 1 with a row vector");
  const int chunk = std::min<int>(n, MLP_LOSS_CHUNK);
  const int n_chunks = (n + chunk - 1) / chunk;
  DeviceGuard dg(c->device);
  if ((r = ensure_mlp_scratch(c, lay, chunk))) return r;
  if ((r = ensure(c, c->mlp_lpart, (size_t)n_chunks * MSE_BLOCKS * 8, "loss partials"))) return r;
  hipStream_t s = (hipStream_t)stream;
  const int dL = lay.d[lay.L];
  float *pre = (float *)c->mlp_pre.p;
  hipError_t e = hipSuccess;
  for (int q = 0; q < n_chunks && e == hipSuccess; ++q) {
    const int k0 = q * chunk, m = std::min(chunk, n - k0);
    // the output layer's pre-activations follow those of the hidden layers, m rows each
    int64_t poff_last = 0;
    for (int l = 0; l < lay.L - 1; ++l) poff_last += (int64_t)m * lay.d[l + 1];
    // without a row vector, chunk q is rows k0 .. k0 + m - 1 of x and t
    const float *xq = rows ? x : x + (int64_t)k0 * lay.d[0];
    const float *tq = rows ? t : t + (int64_t)k0 * dL;
    const int32_t *rq = rows ? rows + k0 : nullptr;
    e = forward_impl(c, net, lay, m, xq, rq, n_total, nullptr, s);
    if (e == hipSuccess)
      e = launch_mse_grad(pre + poff_last, tq, (int64_t)m * dL, dL, rq, n_total, 1.0, nullptr,
                          (double *)c->mlp_lpart.p + (int64_t)q * MSE_BLOCKS, nullptr, c->status, s);
  }
  if (e == hipSuccess)
    e = launch_sum_partials((const double *)c->mlp_lpart.p, (int64_t)n_chunks * MSE_BLOCKS,
                            1.0 / ((double)n * (double)dL), mse_out, s);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_mlp_loss");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_log_hess_target(pcmd_ctx *c, const uint32_t *hess, int32_t n, int32_t nbins, float *out, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (!hess || !out || n < 1 || nbins < 1 || nbins > 1 << 20)
    return fail(c, PCMD_E_INVAL, "pcmd_log_hess_target: bad argument");
  DeviceGuard dg(c->device);
  hipError_t e = launch_log_hess_target(hess, n, nbins, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_log_hess_target");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_surrogate_loglike(pcmd_ctx *c, const float *y, int32_t n, int32_t nbins, const uint32_t *hess_data,
                           double *out, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (!y || !hess_data || !out || n < 1 || nbins < 1 || nbins > 1 << 20)
    return fail(c, PCMD_E_INVAL, "pcmd_surrogate_loglike: bad argument");
  DeviceGuard dg(c->device);
  hipError_t e = launch_surrogate_loglike(y, n, nbins, hess_data, out, c->lnfact64, LNFACT64_N, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_surrogate_loglike");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_gemm_bf16(pcmd_ctx *c, int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t lda, int32_t a_trans,
                   const uint16_t *B, int32_t ldb, int32_t b_trans, float *C, int32_t ldc, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return fail(c, PCMD_E_INVAL, "pcmd_gemm_bf16: bad argument");
  if (lda < (a_trans ? M : K) || ldb < (b_trans ? N : K) || ldc < N)
    return fail(c, PCMD_E_INVAL, "pcmd_gemm_bf16: leading dimension too small");
  DeviceGuard dg(c->device);
  GemmArgs g{};
  g.M = M;
  g.N = N;
  g.K = K;
  g.A = (const __bf16 *)A;
  g.lda = lda;
  g.B = (const __bf16 *)B;
  g.ldb = ldb;
  g.C = C;
  g.ldc = ldc;
  const size_t ws = gemm_workspace_bytes(M, N, K, a_trans != 0, b_trans != 0);
  int r;
  if (ws && (r = ensure(c, c->mlp_ws, ws, "GEMM workspace"))) return r;
  hipError_t e;
  {
    ScopedTimer tm(c, PCMD_TIMER_GEMM, 2.0 * (double)M * (double)N * (double)K, (hipStream_t)stream);
    e = launch_gemm(g, a_trans != 0, b_trans != 0, EPI_STORE, c->mlp_ws.p, c->mlp_ws.n,
                    (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_gemm_bf16");
  c->err.clear();
  return PCMD_OK;
}

}  // extern "C"
