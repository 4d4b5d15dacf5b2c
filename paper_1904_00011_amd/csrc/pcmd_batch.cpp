// Batched evaluation of many parameter points (C ABI): one persistent sampler launch whose tiles
// are balanced across jobs of uneven image size and entry count, per-job launches for the other
// steps, all driven by device descriptor tables so that the launch sequence can be captured once
// into a HIP graph and replayed with new parameters.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "pcmd_ctx.h"
#include "pcmd_device.h"
#include "pcmd_internal.h"

using namespace pcmd;

namespace {

struct JobInfo {
  int E, B, N, npx, K, S, nchunks, pblocks, items, grid;
  int alias_parts;  // 2 when table entries are thinned into two parts, else 1
  int sampler;      // PCMD_SAMPLER_*
  int thin_mode;    // THIN_*
  int nb;           // 64-entry blocks (block-skip and hybrid samplers)
  double cost;
  size_t o_rec, o_thr, o_pc, o_fl, o_part, o_img, o_alias, o_rdesc, o_blk;
};

// Bytes of one job's block-skip tables: [nb] BlockRec, [nb][THR_STRIDE] thresholds, [nb] PtrsConst,
// [nb][SBLK] cumulative thresholds (the layout pcmd_simulate uses).
size_t blk_rec_bytes(int nb) { return (size_t)nb * sizeof(BlockRec); }
size_t blk_thr_bytes(int nb) { return (size_t)nb * THR_STRIDE * 4; }
size_t blk_pc_bytes(int nb) { return (size_t)nb * sizeof(PtrsConst); }
size_t blk_cth_bytes(int nb) { return (size_t)nb * SBLK * 4; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct pcmd_batch_plan {
  uint64_t sig = 0;
  int n_jobs = 0, B = 0, nbins = 0, total_items = 0, wg = 0, order_mode = 0;
  std::vector<JobInfo> info;
  std::vector<int> order;  // sampler table position -> job
  Buf rec, thr, pc, fl, part, F, G, mags, hess, mom, mom_part, ll_part, counters, desc, alias, rdesc, blk;
  void *desc_host = nullptr;
  size_t desc_bytes = 0;
  size_t o_prep = 0, o_samp = 0, o_red = 0, o_conv = 0, o_noise = 0, o_hess = 0, o_ll = 0, o_bprep = 0, o_bsamp = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_desc = nullptr;
  bool desc_pending = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t thin_gen = 0;  // generation of the current call's thinned-entry words
};

namespace pcmd {

// job j's thinned-entry word: k_prep stores the call's generation there when it thins an entry
static uint32_t *thin_word(pcmd_batch_plan *p, int j) { return (uint32_t *)p->counters.p + p->n_jobs + 1 + j; }

static void plan_free_device(pcmd_batch_plan *p) {
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  p->exec = nullptr;
  p->graph = nullptr;
  Buf *bufs[] = {&p->rec, &p->thr, &p->pc, &p->fl, &p->part, &p->F, &p->G, &p->mags, &p->hess, &p->mom, &p->mom_part, &p->ll_part,
                 &p->counters, &p->desc, &p->alias, &p->rdesc, &p->blk};
  for (Buf *b : bufs) release(*b);
  if (p->desc_host) (void)hipHostFree(p->desc_host);
  p->desc_host = nullptr;
  p->desc_bytes = 0;
  p->sig = 0;
}

void batch_destroy(pcmd_ctx *c) {
  pcmd_batch_plan *p = c->batch;
  if (!p) return;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  plan_free_device(p);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_out) (void)hipEventDestroy(p->ev_out);
  if (p->ev_desc) (void)hipEventDestroy(p->ev_desc);
  if (p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
  c->batch = nullptr;
}

static uint64_t fnv(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xFFu;
    h *= 1099511628211ull;
  }
  return h;
}

static int batch_validate(pcmd_ctx *c, int n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *g,
                          const uint32_t *hess_data, const double *mom_data, int mode, double eps,
                          const double *logl_out, const char *who) {
  if (n_jobs < 1 || n_jobs > 65536) return fail(c, PCMD_E_INVAL, "%s: n_jobs %d out of range", who, n_jobs);
  if (!jobs || !g || !hess_data || !logl_out) return fail(c, PCMD_E_INVAL, "%s: null argument", who);
  if (g->nx < 1 || g->ny < 1 || (int64_t)g->nx * g->ny > 65536)
    return fail(c, PCMD_E_INVAL, "%s: grid %d x %d out of range", who, g->nx, g->ny);
  if (!(g->dx > 0.0) || !(g->dy > 0.0) || !isfinite(g->x0) || !isfinite(g->y0))
    return fail(c, PCMD_E_INVAL, "%s: bad grid origin or width", who);
  if (mode < 0 || mode > 2) return fail(c, PCMD_E_INVAL, "%s: bad mode %d", who, mode);
  if (mode == PCMD_LL_POISSON && !(eps > 0.0 && isfinite(eps))) return fail(c, PCMD_E_INVAL, "%s: eps must be > 0", who);
  if (mode != PCMD_LL_POISSON && !mom_data) return fail(c, PCMD_E_INVAL, "%s: data moments needed", who);
  const int B = jobs[0].iso.n_bands;
  for (int j = 0; j < n_jobs; ++j) {
    int r = validate_sim(c, &jobs[j].iso, &jobs[j].obs, who);
    if (r) return r;
    if (jobs[j].iso.n_bands != B) return fail(c, PCMD_E_INVAL, "%s: job %d has %d bands, job 0 has %d", who, j,
                                              jobs[j].iso.n_bands, B);
    if (uses_fft(&jobs[j].obs))
      return fail(c, PCMD_E_UNSUPPORTED, "%s: job %d resolves to the FFT convolution; batches use the direct path", who, j);
  }
  if (g->b_blue < 0 || g->b_blue >= B || g->b_red < 0 || g->b_red >= B || g->b_mag < 0 || g->b_mag >= B)
    return fail(c, PCMD_E_INVAL, "%s: band index out of range", who);
  return PCMD_OK;
}

static int plan_build(pcmd_ctx *c, pcmd_batch_plan *p, int n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *g,
                      uint64_t sig) {
  plan_free_device(p);
  p->n_jobs = n_jobs;
  p->B = jobs[0].iso.n_bands;
  p->nbins = g->nx * g->ny;
  p->wg = c->tune_wg_per_cu;
  p->order_mode = c->tune_order;
  p->info.assign(n_jobs, JobInfo{});
  const int B = p->B, BP = B <= 2 ? 2 : 4;
  size_t n_rec = 0, n_thr = 0, n_pc = 0, n_fl = 0, n_part = 0, n_img = 0, n_alias = 0, n_rdesc = 0, n_blk = 0;
  for (int j = 0; j < n_jobs; ++j) {
    JobInfo &ji = p->info[j];
    ji.E = jobs[j].iso.n_entries;
    ji.B = B;
    ji.N = jobs[j].obs.nim;
    ji.npx = ji.N * ji.N;
    ji.K = jobs[j].obs.psf_k;
    ji.thin_mode = thin_mode_of_split(split_mode_of(&jobs[j].obs));
    ji.alias_parts = ji.thin_mode == THIN_TABLE ? 2 : 1;  // F = 1/2: the halves share one table
    ji.grid = psf_grid_of(&jobs[j].obs);
    // Every batch job keeps both partial streams (unreddened, reddened), so the persistent
    // sampler has one instantiation; a job without a split draws no reddened stars, its second
    // stream holds zeros and the reduction's sums are unchanged (c + 0 = c).
    ji.S = 2;
    ji.nchunks = sample_slices(ji.E, ji.npx);
    ji.pblocks = (ji.npx + 63) / 64;  // one persistent-sampler item = one wave's 64 pixels x one slice
    ji.sampler = jobs[j].obs.sampler;
    ji.nb = superblocks(ji.E);
    // a block-skip job draws everything in its own launch after the persistent sampler
    ji.items = ji.sampler == PCMD_SAMPLER_BLOCK ? 0 : ji.nchunks * ji.pblocks;
    ji.cost = ji.items == 0 ? 0.0
                            : (double)ji.npx * (double)ji.E * (split_mode_of(&jobs[j].obs) == SPLIT_NONE ? 1.0 : 1.3);
    ji.o_rec = n_rec;
    ji.o_thr = n_thr;
    ji.o_pc = n_pc;
    ji.o_fl = n_fl;
    ji.o_part = n_part;
    ji.o_img = n_img;
    ji.o_alias = n_alias;
    ji.o_rdesc = n_rdesc;
    ji.o_blk = n_blk;
    if (ji.sampler != PCMD_SAMPLER_POINT)
      n_blk += align256(blk_rec_bytes(ji.nb) + blk_thr_bytes(ji.nb) + blk_pc_bytes(ji.nb) + blk_cth_bytes(ji.nb));
    n_rec += (rec_bytes(ji.E) + sizeof(EntryRec) - 1) / sizeof(EntryRec);
    n_thr += (size_t)entries_padded(ji.E) * THR_STRIDE;
    n_pc += (size_t)ji.E * 2;
    n_fl += (size_t)ji.E * BP;
    n_part += (size_t)ji.nchunks * ji.S * B * ji.npx;
    n_img += (size_t)B * ji.npx;
    n_alias += (size_t)ji.E * 2 * ALIAS_COLS;
    n_rdesc += (size_t)ji.E;
  }
  p->order.resize(n_jobs);
  std::iota(p->order.begin(), p->order.end(), 0);
  if (p->order_mode == 0)
    std::stable_sort(p->order.begin(), p->order.end(),
                     [&](int a, int b) { return p->info[a].cost > p->info[b].cost; });
  p->total_items = 0;
  for (int j = 0; j < n_jobs; ++j) p->total_items += p->info[p->order[j]].items;
  int r;
  if ((r = ensure(c, p->rec, n_rec * sizeof(EntryRec), "batch entry records"))) return r;
  if ((r = ensure(c, p->thr, n_thr * 4, "batch thresholds"))) return r;
  if ((r = ensure(c, p->pc, n_pc * sizeof(PtrsConst), "batch rejection constants"))) return r;
  if ((r = ensure(c, p->alias, n_alias * 4, "batch alias columns"))) return r;
  if ((r = ensure(c, p->rdesc, n_rdesc * 4, "batch reddened-part descriptors"))) return r;
  if (n_blk && (r = ensure(c, p->blk, n_blk, "batch block tables"))) return r;
  if ((r = ensure(c, p->fl, n_fl * 8, "batch fluxes"))) return r;
  if ((r = ensure(c, p->part, n_part * 4, "batch partial sums"))) return r;
  if ((r = ensure(c, p->F, n_img * 4, "batch images"))) return r;
  if ((r = ensure(c, p->G, n_img * 4, "batch convolved images"))) return r;
  if ((r = ensure(c, p->mags, n_img * 4, "batch magnitudes"))) return r;
  if ((r = ensure(c, p->hess, (size_t)n_jobs * p->nbins * 4, "batch Hess"))) return r;
  if ((r = ensure(c, p->mom, (size_t)n_jobs * 3 * 8, "batch moments"))) return r;
  if ((r = ensure(c, p->mom_part, (size_t)n_jobs * hess_max_blocks() * 3 * 8, "batch moment partials"))) return r;
  if ((r = ensure(c, p->ll_part, (size_t)n_jobs * loglike_blocks(g->nx * g->ny) * 8, "batch likelihood partials")))
    return r;
  // [n_jobs] Hess block counters, the persistent sampler's item counter, [n_jobs] thinned-entry
  // generation words
  if ((r = ensure(c, p->counters, (size_t)(2 * n_jobs + 1) * 4, "batch counters"))) return r;
  hipError_t e = hipMemsetAsync(p->counters.p, 0, (size_t)(2 * n_jobs + 1) * 4, p->stream);  // outside any graph
  if (e != hipSuccess) return hip_fail(c, e, "clearing batch counters");
  size_t o = 0;
  p->o_prep = o;
  o = align256(o + sizeof(PrepArgs) * n_jobs);
  p->o_samp = o;
  o = align256(o + sizeof(BatchSampleJob) * n_jobs);
  p->o_red = o;
  o = align256(o + sizeof(ReduceArgs) * n_jobs);
  p->o_conv = o;
  o = align256(o + sizeof(ConvArgs) * n_jobs);
  p->o_noise = o;
  o = align256(o + sizeof(NoiseArgs) * n_jobs);
  p->o_hess = o;
  o = align256(o + sizeof(HessArgs) * n_jobs);
  p->o_ll = o;
  o = align256(o + sizeof(LoglikeArgs) * n_jobs);
  p->o_bprep = o;
  o = align256(o + sizeof(BlockPrepArgs) * n_jobs);
  p->o_bsamp = o;
  o = align256(o + sizeof(BlockSampleArgs) * n_jobs);
  p->desc_bytes = o;
  if ((r = ensure(c, p->desc, o, "batch descriptors"))) return r;
  e = hipHostMalloc(&p->desc_host, o, hipHostMallocDefault);
  if (e != hipSuccess) {
    p->desc_host = nullptr;
    return fail(c, PCMD_E_NOMEM, "cannot allocate %zu bytes of pinned host memory", o);
  }
  memset(p->desc_host, 0, o);
  p->sig = sig;
  return PCMD_OK;
}

// Write this call's descriptors (pointers, seeds, parameters) into the pinned host blob.
static void fill_descriptors(pcmd_ctx *c, pcmd_batch_plan *p, const pcmd_job *jobs, const pcmd_hess_grid *g,
                             const uint32_t *hess_data, const double *mom_data, int mode, double eps, double *logl_out,
                             uint32_t *hess_out) {
  char *h = (char *)p->desc_host;
  PrepArgs *pa = (PrepArgs *)(h + p->o_prep);
  BatchSampleJob *sa = (BatchSampleJob *)(h + p->o_samp);
  ReduceArgs *ra = (ReduceArgs *)(h + p->o_red);
  ConvArgs *ca = (ConvArgs *)(h + p->o_conv);
  NoiseArgs *na = (NoiseArgs *)(h + p->o_noise);
  HessArgs *ha = (HessArgs *)(h + p->o_hess);
  LoglikeArgs *la = (LoglikeArgs *)(h + p->o_ll);
  BlockPrepArgs *bpa = (BlockPrepArgs *)(h + p->o_bprep);
  BlockSampleArgs *bsa = (BlockSampleArgs *)(h + p->o_bsamp);
  const int B = p->B, BP = B <= 2 ? 2 : 4;
  // a new generation per call: a job's word equals it only if this call's k_prep thinned one of
  // its entries (a stale match would only cost the sampler a scan of the group flags)
  ++p->thin_gen;
  int item0 = 0;
  std::vector<int> first_item(p->n_jobs, 0);
  for (int t = 0; t < p->n_jobs; ++t) {
    first_item[p->order[t]] = item0;
    item0 += p->info[p->order[t]].items;
  }
  for (int j = 0; j < p->n_jobs; ++j) {
    const JobInfo &ji = p->info[j];
    const pcmd_obs *o = &jobs[j].obs;
    EntryRec *rec = (EntryRec *)p->rec.p + ji.o_rec;
    uint32_t *thr = (uint32_t *)p->thr.p + ji.o_thr;
    PtrsConst *pc = (PtrsConst *)p->pc.p + ji.o_pc;
    double *fl = (double *)p->fl.p + ji.o_fl;
    float *part = (float *)p->part.p + ji.o_part;
    float *F = (float *)p->F.p + ji.o_img;
    float *G = (float *)p->G.p + ji.o_img;
    float *mags = (float *)p->mags.p + ji.o_img;
    const uint32_t k0 = (uint32_t)(o->seed & 0xFFFFFFFFu), k1 = (uint32_t)(o->seed >> 32);
    GroupRec *grp = (GroupRec *)(rec + entries_padded(ji.E));
    const int sm = split_mode_of(&jobs[j].obs);
    // block-skip tables (block and hybrid samplers), as pcmd_simulate lays them out
    BlockPrepArgs bp;
    memset(&bp, 0, sizeof bp);
    BlockSampleArgs bs;
    memset(&bs, 0, sizeof bs);
    if (ji.sampler != PCMD_SAMPLER_POINT) {
      char *base = (char *)p->blk.p + ji.o_blk;
      const size_t r_b = blk_rec_bytes(ji.nb), t_b = blk_thr_bytes(ji.nb), c_b = blk_pc_bytes(ji.nb);
      bp = BlockPrepArgs{ji.E,
                         B,
                         BP,
                         ji.nb,
                         jobs[j].iso.lam,
                         jobs[j].iso.flux,
                         (BlockRec *)base,
                         (uint32_t *)(base + r_b),
                         base + r_b + t_b,
                         (uint32_t *)(base + r_b + t_b + c_b),
                         fl,
                         c->status,
                         ji.sampler == PCMD_SAMPLER_HYBRID ? 1 : 0};
      bs.E = ji.E;
      bs.B = B;
      bs.BP = BP;
      bs.npx = ji.npx;
      bs.nb = ji.nb;
      bs.nchunks = ji.nchunks;
      bs.S = ji.S;
      bs.k0 = k0;
      bs.k1 = k1;
      bs.split_mode = sm;
      bs.split_q = split_q_of(o);
      bs.brec = bp.brec;
      bs.thr = bp.thr;
      bs.pc = bp.pc;
      bs.cth = bp.cth;
      bs.fl64 = fl;
      bs.part = part;
      bs.status = c->status;
      bs.lnfact = c->lnfact;
      bs.accumulate = ji.sampler == PCMD_SAMPLER_HYBRID ? 1 : 0;  // hybrid: after the per-point pass
    }
    bpa[j] = bp;
    bsa[j] = bs;
    pa[j] = PrepArgs{ji.E,
                     B,
                     BP,
                     jobs[j].iso.lam,
                     jobs[j].iso.flux,
                     rec,
                     grp,
                     thr,
                     pc,
                     fl,
                     c->status,
                     (uint32_t *)p->alias.p + ji.o_alias,
                     ji.sampler == PCMD_SAMPLER_HYBRID ? bp.brec : nullptr,
                     thin_mode_of_split(sm),
                     jobs[j].obs.dust_frac,
                     (uint32_t *)p->rdesc.p + ji.o_rdesc,
                     thin_word(p, j),
                     p->thin_gen};
    ReduceArgs rr;
    memset(&rr, 0, sizeof rr);
    rr.B = B;
    rr.npx = ji.npx;
    rr.nchunks = ji.nchunks;
    rr.S = ji.S;
    rr.part = part;
    rr.F = F;
    rr.dist = pow(10.0, -0.4 * o->dmod);
    rr.dust_model = o->dust_model;
    rr.dust_mu = o->dust_mu;
    rr.dust_sigma = o->dust_sigma;
    for (int b = 0; b < PCMD_MAX_BANDS; ++b) rr.dust_R[b] = b < B ? o->dust_R[b] : 0.0;
    rr.k0 = k0;
    rr.k1 = k1;
    ra[j] = rr;
    ca[j] = ConvArgs{B, ji.N, ji.K, F, o->psf, G, c->status, psf_grid_of(o)};
    NoiseArgs nn;
    memset(&nn, 0, sizeof nn);
    nn.B = B;
    nn.npx = ji.npx;
    nn.G = ji.K > 1 ? G : F;
    nn.mags = mags;
    nn.noise_model = o->noise_model;
    for (int b = 0; b < PCMD_MAX_BANDS; ++b) {
      nn.sigma[b] = b < B ? o->noise_sigma_mag[b] : 0.0;
      nn.exptime[b] = b < B ? o->exptime[b] : 1.0;
      nn.zp[b] = b < B ? o->zp[b] : 0.0;
      nn.sky[b] = b < B ? o->sky[b] : 0.0;
    }
    nn.k0 = k0;
    nn.k1 = k1;
    na[j] = nn;
    HessArgs hh;
    memset(&hh, 0, sizeof hh);
    hh.mags = mags;
    hh.npx = ji.npx;
    hh.x0 = g->x0;
    hh.dx = g->dx;
    hh.y0 = g->y0;
    hh.dy = g->dy;
    hh.nx = g->nx;
    hh.ny = g->ny;
    hh.bb = g->b_blue;
    hh.br = g->b_red;
    hh.bm = g->b_mag;
    hh.hess = hess_out ? hess_out + (size_t)j * p->nbins : (uint32_t *)p->hess.p + (size_t)j * p->nbins;
    hh.mom_part = (double *)p->mom_part.p + (size_t)j * hess_max_blocks() * 3;
    hh.counter = (uint32_t *)p->counters.p + j;
    hh.moments = (double *)p->mom.p + (size_t)j * 3;
    hh.use_lds = hess_use_lds(p->nbins);
    ha[j] = hh;
    la[j] = LoglikeArgs{hh.hess, hess_data,    p->nbins,    mode, hh.moments, mom_data, eps, logl_out + j,
                        (double *)p->ll_part.p + (size_t)j * loglike_blocks(p->nbins), 0, c->lnfact64};
  }
  for (int t = 0; t < p->n_jobs; ++t) {
    const int j = p->order[t];
    BatchSampleJob bj;
    memset(&bj, 0, sizeof bj);
    const JobInfo &ji = p->info[j];
    const pcmd_obs *o = &jobs[j].obs;
    SampleArgs &s = bj.a;
    s.E = ji.E;
    s.B = B;
    s.BP = BP;
    s.npx = ji.npx;
    s.nchunks = ji.nchunks;
    s.S = ji.S;
    s.k0 = (uint32_t)(o->seed & 0xFFFFFFFFu);
    s.k1 = (uint32_t)(o->seed >> 32);
    s.split_mode = split_mode_of(o);
    s.split_q = split_q_of(o);
    s.rec = (EntryRec *)p->rec.p + ji.o_rec;
    s.grp = (const GroupRec *)(s.rec + entries_padded(ji.E));
    s.thr = (uint32_t *)p->thr.p + ji.o_thr;
    s.pc = (PtrsConst *)p->pc.p + ji.o_pc;
    s.part = (float *)p->part.p + ji.o_part;
    s.status = c->status;
    s.lnfact = c->lnfact;
    s.alias = (const uint32_t *)p->alias.p + ji.o_alias;
    s.rdesc = (const uint32_t *)p->rdesc.p + ji.o_rdesc;
    s.thin_seen = thin_word(p, j);
    s.gen = p->thin_gen;
    bj.item0 = first_item[j];
    bj.items = ji.items;
    bj.pblocks = ji.pblocks;
    sa[t] = bj;
  }
}

// Queue the whole batch on stream s (eagerly, or into a graph under capture).
static hipError_t enqueue(pcmd_ctx *c, pcmd_batch_plan *p, hipStream_t s) {
  char *d = (char *)p->desc.p;
  const PrepArgs *pa = (const PrepArgs *)(d + p->o_prep);
  const BatchSampleJob *sa = (const BatchSampleJob *)(d + p->o_samp);
  const ReduceArgs *ra = (const ReduceArgs *)(d + p->o_red);
  const ConvArgs *ca = (const ConvArgs *)(d + p->o_conv);
  const NoiseArgs *na = (const NoiseArgs *)(d + p->o_noise);
  const HessArgs *ha = (const HessArgs *)(d + p->o_hess);
  const LoglikeArgs *la = (const LoglikeArgs *)(d + p->o_ll);
  const BlockPrepArgs *bpa = (const BlockPrepArgs *)(d + p->o_bprep);
  const BlockSampleArgs *bsa = (const BlockSampleArgs *)(d + p->o_bsamp);
  uint32_t *persist = (uint32_t *)p->counters.p + p->n_jobs;
  hipError_t e = hipSuccess;
  for (int j = 0; j < p->n_jobs && e == hipSuccess; ++j) {
    const JobInfo &ji = p->info[j];
    // block tables first: the hybrid's per-point tables leave out the blocks the block rule draws
    if (ji.sampler != PCMD_SAMPLER_POINT) e = launch_prep_block_job(bpa, j, ji.nb, s);
    if (e == hipSuccess && ji.sampler != PCMD_SAMPLER_BLOCK) {
      e = launch_prep_job(pa, j, ji.E, s);
      if (e == hipSuccess) e = launch_prep_alias_job(pa, j, ji.E, ji.alias_parts, s);
    }
  }
  if (e == hipSuccess) e = launch_reset_counter(persist, s);
  if (e == hipSuccess)
    e = launch_sample_persistent(sa, p->n_jobs, p->total_items, p->B, persist, c->n_cu * p->wg, s);
  // then, in the order pcmd_simulate takes: the thinned entries of F = 1/2 jobs, added to the
  // per-point partials (a launch per job; a job whose k_prep thinned nothing returns at once),
  // and the block-rule draws, stored (block sampler) or added (hybrid)
  for (int t = 0; t < p->n_jobs && e == hipSuccess; ++t) {
    const int j = p->order[t];
    const JobInfo &ji = p->info[j];
    if (ji.items > 0 && ji.thin_mode == THIN_HALF_HIGH) e = launch_sample_thin_job(sa, t, ji.B, ji.npx, ji.nchunks, s);
  }
  for (int j = 0; j < p->n_jobs && e == hipSuccess; ++j) {
    const JobInfo &ji = p->info[j];
    if (ji.sampler != PCMD_SAMPLER_POINT) e = launch_sample_block_job(bsa, j, ji.B, ji.npx, ji.nchunks, s);
  }
  for (int j = 0; j < p->n_jobs && e == hipSuccess; ++j) {
    const JobInfo &ji = p->info[j];
    e = launch_reduce_job(ra, j, ji.npx, ji.B, s);
    if (e == hipSuccess && ji.K > 1) e = launch_conv_direct_job(ca, j, ji.B, ji.N, ji.K, ji.grid, s);
    if (e == hipSuccess) e = launch_noise_mag_job(na, j, ji.npx, s);
  }
  for (int j = 0; j < p->n_jobs && e == hipSuccess; ++j) {
    e = launch_hess_clear_job(ha, j, p->nbins, s);
    if (e == hipSuccess) e = launch_hess_job(ha, j, p->info[j].npx, p->nbins, s);
  }
  if (e == hipSuccess) e = launch_loglike_jobs(la, p->n_jobs, p->nbins, s);
  return e;
}

static uint64_t batch_signature(pcmd_ctx *c, int n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *g) {
  uint64_t h = 1469598103934665603ull;
  h = fnv(h, (uint64_t)n_jobs);
  h = fnv(h, (uint64_t)jobs[0].iso.n_bands);
  h = fnv(h, ((uint64_t)g->nx << 32) | (uint32_t)g->ny);
  h = fnv(h, ((uint64_t)c->tune_wg_per_cu << 32) | (uint32_t)c->tune_order);
  for (int j = 0; j < n_jobs; ++j) {
    // the split mode fixes the plan's alias rows (a thinned job builds its reddened parts' tables
    // too) and with them the captured launches, so every mode is part of the signature
    const int sm = split_mode_of(&jobs[j].obs);
    h = fnv(h, ((uint64_t)jobs[j].iso.n_entries << 32) | (uint32_t)jobs[j].obs.nim);
    h = fnv(h, ((uint64_t)jobs[j].obs.psf_k << 32) | (uint32_t)sm);
    h = fnv(h, ((uint64_t)jobs[j].obs.sampler << 32) | (uint32_t)psf_grid_of(&jobs[j].obs));
  }
  return h;
}

static int batch_run_impl(pcmd_ctx *c, int n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *g,
                          const uint32_t *hess_data, const double *mom_data, int mode, double eps, double *logl_out,
                          uint32_t *hess_out, int use_graph, hipStream_t caller) {
  if (!c->batch) {
    c->batch = new pcmd_batch_plan();
    pcmd_batch_plan *p = c->batch;
    if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_desc, hipEventDisableTiming) != hipSuccess) {
      batch_destroy(c);
      return fail(c, PCMD_E_HIP, "cannot create the batch stream and events");
    }
  }
  pcmd_batch_plan *p = c->batch;
  const uint64_t sig = batch_signature(c, n_jobs, jobs, g);
  int r;
  if (sig != p->sig) {
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(c, e, "batch stream");
    p->desc_pending = false;
    if ((r = plan_build(c, p, n_jobs, jobs, g, sig))) {
      plan_free_device(p);
      return r;
    }
  }
  // the previous call's descriptor upload must have left the pinned blob before it is rewritten
  if (p->desc_pending) {
    hipError_t e = hipEventSynchronize(p->ev_desc);
    if (e != hipSuccess) return hip_fail(c, e, "batch descriptors");
    p->desc_pending = false;
  }
  fill_descriptors(c, p, jobs, g, hess_data, mom_data, mode, eps, logl_out, hess_out);
  hipError_t e = hipEventRecord(p->ev_in, caller);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->ev_in, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(p->desc.p, p->desc_host, p->desc_bytes, hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) e = hipEventRecord(p->ev_desc, p->stream);
  if (e != hipSuccess) return hip_fail(c, e, "batch descriptor upload");
  p->desc_pending = true;
  double draws = 0.0;
  for (const JobInfo &ji : p->info) draws += (double)ji.npx * (double)ji.E;
  {
    ScopedTimer tm(c, PCMD_TIMER_BATCH, draws, p->stream);
    if (use_graph) {
      if (!p->exec) {
        const bool timing = c->timing;
        c->timing = false;
        e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          hipError_t e2 = enqueue(c, p, p->stream);
          e = hipStreamEndCapture(p->stream, &p->graph);
          if (e == hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
        c->timing = timing;
        if (e != hipSuccess) {
          if (p->graph) (void)hipGraphDestroy(p->graph);
          p->graph = nullptr;
          p->exec = nullptr;
          return hip_fail(c, e, "capturing the batch graph");
        }
      }
      e = hipGraphLaunch(p->exec, p->stream);
    } else {
      e = enqueue(c, p, p->stream);
    }
  }
  if (e != hipSuccess) return hip_fail(c, e, "batch launch");
  e = hipEventRecord(p->ev_out, p->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(caller, p->ev_out, 0);
  if (e != hipSuccess) return hip_fail(c, e, "batch completion event");
  return PCMD_OK;
}

}  // namespace pcmd

extern "C" {

int pcmd_batch_run(pcmd_ctx *c, int32_t n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *grid,
                   const uint32_t *hess_data, const double *mom_data, int32_t mode, double eps, double *logl_out,
                   uint32_t *hess_out, int32_t use_graph, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  int r = batch_validate(c, n_jobs, jobs, grid, hess_data, mom_data, mode, eps, logl_out, "pcmd_batch_run");
  if (r) return r;
  DeviceGuard dg(c->device);
  r = batch_run_impl(c, n_jobs, jobs, grid, hess_data, mom_data, mode, eps, logl_out, hess_out, use_graph,
                     (hipStream_t)stream);
  if (r == PCMD_OK) c->err.clear();
  return r;
}

int pcmd_batch_set_tuning(pcmd_ctx *c, const pcmd_batch_tuning *t) {
  if (!c) return PCMD_E_INVAL;
  if (!t || t->wg_per_cu < 1 || t->wg_per_cu > 8 || t->order < 0 || t->order > 1)
    return fail(c, PCMD_E_INVAL, "pcmd_batch_set_tuning: wg_per_cu must be 1..8 and order 0 or 1");
  c->tune_wg_per_cu = t->wg_per_cu;
  c->tune_order = t->order;
  c->err.clear();
  return PCMD_OK;
}

int pcmd_batch_get_tuning(pcmd_ctx *c, pcmd_batch_tuning *t) {
  if (!c || !t) return PCMD_E_INVAL;
  t->wg_per_cu = c->tune_wg_per_cu;
  t->order = c->tune_order;
  return PCMD_OK;
}

int pcmd_batch_autotune(pcmd_ctx *c, int32_t n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *grid,
                        const uint32_t *hess_data, const double *mom_data, int32_t mode, double eps, double *logl_out,
                        pcmd_batch_tuning *best, double *ms_out, int32_t *n_candidates, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  int r = batch_validate(c, n_jobs, jobs, grid, hess_data, mom_data, mode, eps, logl_out, "pcmd_batch_autotune");
  if (r) return r;
  if (!best) return fail(c, PCMD_E_INVAL, "pcmd_batch_autotune: null best");
  DeviceGuard dg(c->device);
  static const int WG[] = {1, 2, 4, 8};
  const int ncand = 8;
  hipStream_t s = (hipStream_t)stream;
  const int save_wg = c->tune_wg_per_cu, save_order = c->tune_order;
  const bool save_timing = c->timing;
  c->timing = false;
  double best_ms = 1e300;
  pcmd_batch_tuning bt{save_wg, save_order};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    c->timing = save_timing;
    return fail(c, PCMD_E_HIP, "pcmd_batch_autotune: events");
  }
  for (int k = 0; k < ncand && r == PCMD_OK; ++k) {
    c->tune_wg_per_cu = WG[k / 2];
    c->tune_order = k % 2;
    // first run builds the plan for this schedule (allocation), second run is timed
    r = batch_run_impl(c, n_jobs, jobs, grid, hess_data, mom_data, mode, eps, logl_out, nullptr, 0, s);
    if (r) break;
    hipError_t e = hipEventRecord(e0, s);
    if (e == hipSuccess)
      r = batch_run_impl(c, n_jobs, jobs, grid, hess_data, mom_data, mode, eps, logl_out, nullptr, 0, s);
    if (r) break;
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      r = hip_fail(c, e, "pcmd_batch_autotune timing");
      break;
    }
    if (ms_out) ms_out[k] = ms;
    if (ms < best_ms) {
      best_ms = ms;
      bt = pcmd_batch_tuning{c->tune_wg_per_cu, c->tune_order};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->timing = save_timing;
  if (r) {
    c->tune_wg_per_cu = save_wg;
    c->tune_order = save_order;
    return r;
  }
  c->tune_wg_per_cu = bt.wg_per_cu;
  c->tune_order = bt.order;
  *best = bt;
  if (n_candidates) *n_candidates = ncand;
  c->err.clear();
  return PCMD_OK;
}

}  // extern "C"
