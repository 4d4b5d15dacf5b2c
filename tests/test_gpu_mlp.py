"""Surrogate network on BF16 MFMA against the oracle network (FP64 with the same BF16 roundings)."""
import numpy as np
import pytest

import synth_inputs as si
from oracle import mlp as om

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1904_00011_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _bf16_tensor(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.device("cuda")).to(torch.bfloat16)


# the last two split K over several blocks (ragged final split) and sum the parts in order
@pytest.mark.parametrize("M,N,K", [(70, 45, 37), (128, 64, 512), (1, 1, 1), (200, 130, 12), (256, 200, 3000),
                                   (130, 70, 1000)])
@pytest.mark.parametrize("at,bt", [(False, False), (True, True), (True, False), (False, True)])
def test_gemm_layouts_against_fp64(ctx, M, N, K, at, bt):
    import torch
    r = np.random.default_rng(M * 7 + N + K)
    A = om.bf16_round(r.normal(size=(M, K)).astype(np.float32)).astype(np.float64)
    B = om.bf16_round(r.normal(size=(N, K)).astype(np.float32)).astype(np.float64)
    Ad = _bf16_tensor(A.T.copy() if at else A)
    Bd = _bf16_tensor(B.T.copy() if bt else B)
    Cd = torch.full((M, N), float("nan"), dtype=torch.float32, device=torch.device("cuda"))
    print(f"[case] gemm M={M} N={N} K={K} at={at} bt={bt}", flush=True)
    ctx.gemm_bf16(Ad, Bd, Cd, a_trans=at, b_trans=bt)
    ctx.sync()
    ref = A @ B.T
    got = Cd.cpu().numpy().astype(np.float64)
    scale = np.sqrt(K) * 1.0
    assert np.max(np.abs(got - ref)) <= 1e-5 * scale + 1e-6


def _net(ctx, dims, seed):
    from paper_1904_00011_amd.surrogate import SurrogateNet
    master = si.mlp_init(dims, seed)
    return SurrogateNet(ctx, dims, master), master.astype(np.float64)


def test_forward_against_oracle(ctx):
    import torch
    dims = (12, 64, 96, 100)
    net, master = _net(ctx, dims, 3)
    r = np.random.default_rng(4)
    x = r.uniform(-1, 1, (37, 12)).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda())
    ctx.sync()
    yo, _ = om.forward(master.astype(np.float32).astype(np.float64), dims, x)
    got = y.cpu().numpy()
    assert np.max(np.abs(got - yo)) <= 2e-3 * np.max(np.abs(yo))


@pytest.mark.parametrize("n", [53, 600])  # 600: the weight gradients split the batch over two blocks
def test_gradients_against_oracle(ctx, n):
    import torch
    dims = (12, 64, 96, 100)
    net, master = _net(ctx, dims, 5)
    r = np.random.default_rng(6)
    x = r.uniform(-1, 1, (n, 12)).astype(np.float32)
    t = r.normal(0, 1, (n, 100)).astype(np.float32)
    dev = torch.device("cuda")
    grad = torch.empty(net.n_params, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    net.train_step(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev), 0.0, loss_out=loss, grad_out=grad,
                   apply_update=False)
    ctx.sync()
    lo, go = om.loss_and_grad(master.astype(np.float32).astype(np.float64), dims, x, t)
    assert float(loss.item()) == pytest.approx(lo, rel=1e-4)
    g = grad.cpu().numpy().astype(np.float64)
    o = 0
    for l in range(len(dims) - 1):
        n = dims[l + 1] * dims[l] + dims[l + 1]
        gl, ol_ = g[o:o + n], go[o:o + n]
        print(f"[case] grad layer {l} max|g|={np.max(np.abs(ol_)):.3e} maxdiff={np.max(np.abs(gl - ol_)):.3e}", flush=True)
        assert np.max(np.abs(gl - ol_)) <= 1e-2 * np.max(np.abs(ol_))
        assert np.corrcoef(gl, ol_)[0, 1] > 0.9999
        o += n


def test_adam_step_against_oracle(ctx):
    import torch
    dims = (12, 32, 40)
    net, master = _net(ctx, dims, 7)
    r = np.random.default_rng(8)
    x = r.uniform(-1, 1, (16, 12)).astype(np.float32)
    t = r.normal(0, 1, (16, 40)).astype(np.float32)
    dev = torch.device("cuda")
    lr = 1e-3
    net.train_step(torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev), lr)
    ctx.sync()
    m32 = master.astype(np.float32).astype(np.float64)
    _, go = om.loss_and_grad(m32, dims, x, t)
    new, _, _ = om.adam_update(m32, go, np.zeros_like(go), np.zeros_like(go), 1, lr)
    got = net.master.cpu().numpy().astype(np.float64)
    big = np.abs(go) > 1e-5          # the first Adam step is lr * sign(g) wherever |g| >> eps
    assert np.max(np.abs(got - new)[big]) <= 1e-3 * lr + 1e-7
    assert np.max(np.abs(got - m32)) <= lr * (1 + 1e-3)
    # BF16 shadows follow the master weights
    w = net.w.float().cpu().numpy()
    assert np.array_equal(w[:32 * 12], om.bf16_round(got[:32 * 12].astype(np.float32)))


def test_training_reduces_loss(ctx):
    import torch
    dims = (12, 128, 128, 64)
    net, _ = _net(ctx, dims, 9)
    r = np.random.default_rng(10)
    P = r.normal(size=(12, 64))
    x = r.uniform(-1, 1, (512, 12)).astype(np.float32)
    t = np.sin(x @ P).astype(np.float32)
    dev = torch.device("cuda")
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    first = None
    for k in range(400):
        net.train_step(xd, td, 3e-3, loss_out=loss)
        if k == 0:
            ctx.sync()
            first = float(loss.item())
    ctx.sync()
    last = float(loss.item())
    print(f"[case] training loss {first:.4f} -> {last:.4f}", flush=True)
    assert last < 0.1 * first


def test_surrogate_loglike_against_oracle(ctx):
    import torch
    r = np.random.default_rng(11)
    y = r.normal(-9, 1, (5, 10000)).astype(np.float32)
    d = r.poisson(2.0, 10000)
    dev = torch.device("cuda")
    out = torch.empty(5, dtype=torch.float64, device=dev)
    ctx.surrogate_loglike(torch.from_numpy(y).to(dev), torch.from_numpy(d.astype(np.int32)).to(dev), out)
    ctx.sync()
    for k in range(5):
        assert out[k].item() == pytest.approx(om.surrogate_loglike(y[k], d), rel=1e-9)


def test_backward_with_rows_matches_the_gathered_batch(ctx):
    """pcmd_mlp_backward on rows of a set gives the gradient and loss of the explicitly gathered
    batch (the same kernels on the same values, so bit-identical), and backward + adam equals the
    fused training step."""
    import torch
    dims = (12, 64, 96, 100)
    dev = torch.device("cuda")
    r = np.random.default_rng(21)
    X = r.uniform(-1, 1, (300, 12)).astype(np.float32)
    T = r.normal(0, 1, (300, 100)).astype(np.float32)
    rows = r.integers(0, 300, 77).astype(np.int32)
    Xd, Td = torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev)
    rows_d = torch.from_numpy(rows).to(dev)
    net_a, master = _net(ctx, dims, 22)
    net_b, _ = _net(ctx, dims, 22)
    ga = torch.empty(net_a.n_params, dtype=torch.float32, device=dev)
    gb = torch.empty_like(ga)
    la = torch.empty(1, dtype=torch.float32, device=dev)
    lb = torch.empty_like(la)
    ctx.mlp_backward(net_a.struct, Xd, Td, ga, rows=rows_d, loss_out=la)
    xb = torch.from_numpy(X[rows]).to(dev)
    tb = torch.from_numpy(T[rows]).to(dev)
    net_b.train_step(xb, tb, 0.0, loss_out=lb, grad_out=gb, apply_update=False)
    ctx.sync()
    assert torch.equal(ga, gb) and torch.equal(la, lb)
    lo, go = om.loss_and_grad(master.astype(np.float32).astype(np.float64), dims, X[rows], T[rows])
    assert float(la.item()) == pytest.approx(lo, rel=1e-4)
    # backward + adam (split) == train_step (fused)
    net_a.train_step_rows(Xd, Td, rows_d, 1e-3, ga)
    net_b.train_step(xb, tb, 1e-3)
    ctx.sync()
    assert torch.equal(net_a.master, net_b.master)
    assert torch.equal(net_a.m, net_b.m) and torch.equal(net_a.v, net_b.v)
    assert torch.equal(net_a.w, net_b.w) and torch.equal(net_a.wt, net_b.wt)


def test_backward_flags_a_row_outside_the_set(ctx):
    """A row index outside [0, n_total) is read as row 0 and reported by pcmd_sync."""
    import torch
    import paper_1904_00011_amd as P
    dims = (12, 32, 40)
    dev = torch.device("cuda")
    net, _ = _net(ctx, dims, 23)
    X = torch.zeros((10, 12), dtype=torch.float32, device=dev)
    T = torch.zeros((10, 40), dtype=torch.float32, device=dev)
    rows = torch.tensor([0, 3, 10, 2], dtype=torch.int32, device=dev)
    g = torch.empty(net.n_params, dtype=torch.float32, device=dev)
    ctx.mlp_backward(net.struct, X, T, g, rows=rows)
    with pytest.raises(P.PcmdError):
        ctx.sync()
    ctx.sync()  # the finding was cleared


@pytest.mark.parametrize("n,use_rows", [(2500, False), (1024, False), (700, True)])
def test_set_loss_against_oracle(ctx, n, use_rows):
    """pcmd_mlp_loss over a set of several 1,024-row forward passes (ragged last one) against the
    oracle network's mean squared error."""
    import torch
    dims = (12, 64, 96, 100)
    dev = torch.device("cuda")
    net, master = _net(ctx, dims, 24)
    r = np.random.default_rng(25 + n)
    N = 2000 if use_rows else n
    X = r.uniform(-1, 1, (N, 12)).astype(np.float32)
    T = r.normal(0, 1, (N, 100)).astype(np.float32)
    rows = r.integers(0, N, n).astype(np.int32) if use_rows else np.arange(n, dtype=np.int32)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    Xd, Td = torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev)
    net.loss(Xd, Td, out, rows=torch.from_numpy(rows).to(dev) if use_rows else None)
    ctx.sync()
    yo, _ = om.forward(master.astype(np.float32).astype(np.float64), dims, X[rows])
    mo = om.mse(yo, T[rows])
    print(f"[case] set loss n={n} rows={use_rows}: GPU {float(out.item()):.8f} oracle {mo:.8f}", flush=True)
    assert float(out.item()) == pytest.approx(mo, rel=1e-4)


def test_log_hess_target_against_oracle(ctx):
    import torch
    r = np.random.default_rng(26)
    h = r.poisson(r.gamma(0.3, 20.0, size=(6, 10000))).astype(np.int32)
    h[3] = 0
    out = torch.empty((6, 10000), dtype=torch.float32, device=torch.device("cuda"))
    ctx.log_hess_target(torch.from_numpy(h).cuda(), out)
    ctx.sync()
    to = om.log_hess_target(h)
    got = out.cpu().numpy().astype(np.float64)
    # FP64 on both sides, one rounding to FP32 on the GPU
    assert np.max(np.abs(got - to) / np.abs(to)) <= 2 ** -24 * 1.01


def test_configured_network_against_oracle(ctx):
    """The surrogate's own shape, 12 -> 4 x 512 -> 10,000: forward pass and one gradient on a small
    batch against the oracle network."""
    import torch
    dims = (12, 512, 512, 512, 512, 10000)
    dev = torch.device("cuda")
    net, master = _net(ctx, dims, 27)
    r = np.random.default_rng(28)
    n = 24
    x = r.uniform(-1, 1, (n, 12)).astype(np.float32)
    t = r.normal(-9, 1, (n, 10000)).astype(np.float32)
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(t).to(dev)
    y = net.forward(xd)
    grad = torch.empty(net.n_params, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    net.train_step(xd, td, 0.0, loss_out=loss, grad_out=grad, apply_update=False)
    ctx.sync()
    m32 = master.astype(np.float32).astype(np.float64)
    yo, _ = om.forward(m32, dims, x)
    ey = np.max(np.abs(y.cpu().numpy() - yo)) / np.max(np.abs(yo))
    lo, go = om.loss_and_grad(m32, dims, x, t)
    g = grad.cpu().numpy().astype(np.float64)
    print(f"[case] configured network: forward rel err {ey:.2e}, loss GPU {float(loss.item()):.6f} oracle {lo:.6f}",
          flush=True)
    assert ey <= 2e-3
    assert float(loss.item()) == pytest.approx(lo, rel=1e-4)
    o = 0
    for l in range(len(dims) - 1):
        k = dims[l + 1] * dims[l] + dims[l + 1]
        gl, ol_ = g[o:o + k], go[o:o + k]
        err = np.max(np.abs(gl - ol_)) / np.max(np.abs(ol_))
        print(f"[case] configured network layer {l}: max|g| {np.max(np.abs(ol_)):.3e} rel err {err:.2e} "
              f"corr {np.corrcoef(gl, ol_)[0, 1]:.6f}", flush=True)
        assert err <= 1e-2
        assert np.corrcoef(gl, ol_)[0, 1] > 0.9999
        o += k


@pytest.mark.parametrize("M,N,K", [(4500, 2100, 100), (4096, 10000, 512)])
def test_gemm_tall_tiles_against_fp64(ctx, M, N, K):
    """Products large enough for the 256-row block tiles (ragged in M and N for the first):
    sampled rows against FP64."""
    import torch
    r = np.random.default_rng(M + N + K)
    A = om.bf16_round(r.normal(size=(M, K)).astype(np.float32)).astype(np.float64)
    B = om.bf16_round(r.normal(size=(N, K)).astype(np.float32)).astype(np.float64)
    Cd = torch.full((M, N), float("nan"), dtype=torch.float32, device=torch.device("cuda"))
    print(f"[case] gemm tall M={M} N={N} K={K}", flush=True)
    ctx.gemm_bf16(_bf16_tensor(A), _bf16_tensor(B), Cd)
    ctx.sync()
    rows = np.unique(np.concatenate([r.integers(0, M, 200), [0, 255, 256, M - 1]]))
    got = Cd.cpu().numpy()[rows].astype(np.float64)
    ref = A[rows] @ B.T
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(got - ref)) <= 1e-5 * np.sqrt(K) + 1e-6


def test_configured_network_forward_at_a_large_batch(ctx):
    """The configured network's forward pass at a batch of 4,100 (its 10,000-wide output layer on
    the 256-row tiles, ragged last tile): sampled rows against the oracle network."""
    import torch
    dims = (12, 512, 512, 512, 512, 10000)
    net, master = _net(ctx, dims, 31)
    r = np.random.default_rng(32)
    x = r.uniform(-1, 1, (4100, 12)).astype(np.float32)
    y = net.forward(torch.from_numpy(x).cuda())
    ctx.sync()
    rows = np.unique(np.concatenate([r.integers(0, 4100, 48), [0, 4095, 4096, 4099]]))
    yo, _ = om.forward(master.astype(np.float32).astype(np.float64), dims, x[rows])
    got = y.cpu().numpy()[rows]
    err = np.max(np.abs(got - yo)) / np.max(np.abs(yo))
    print(f"[case] configured network forward at 4100: rel err {err:.2e}", flush=True)
    assert err <= 2e-3
