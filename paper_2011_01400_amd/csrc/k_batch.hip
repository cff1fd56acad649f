// Batched form: several cells of uneven basis / auxiliary size, every
// (cell, q, w) job of a whole pass captured into one hipGraph and replayed
// with a single launch.  Each cell runs on a stream of its own inside the
// capture (fork/join through events), so the small kernels of different cells
// overlap on the device.  Before capture an autotuner times the response
// kernel of every cell over its tile choices (frequencies per workgroup, K
// split count) and keeps the fastest.
#include <algorithm>
#include <climits>
#include <cmath>
#include <new>
#include <vector>

#include "lrigw_internal.h"

// relative time by which a later tuning candidate must beat the best so far
#define TUNE_MARGIN 0.02

struct lrigw_batch {
  std::vector<lrigw_batch_cell> cells;
  hipStream_t stream = nullptr;
  std::vector<hipStream_t> cs;
  std::vector<hipStream_t> saved;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> nw, splits;
  std::vector<double> ms;
  long long launches = 0;
};

// Time the response kernel of one q for every (frequencies per workgroup,
// split) candidate and, in the split-BF16 forms, the self-energy kernel for
// every variant; keep the fastest.  Runs before capture.
static int autotune_chi0(lrigw_ctx *c, const lrigw_batch_cell &cell, int *nw_out, int *S_out, double *ms_out) {
  const Dims &d = c->d;
  hipStream_t s = c->stream;
  const int q = d.n_k > 1 ? 1 : 0;
  LRIGW_TRY(run_build_M(c, q, 0, cell.H, cell.evec, c->d_M));
  const int nw0 = c->chi_nw, S0 = c->chi_splits;
  std::vector<int> nws = {chi0_default_nw(c->precision), chi0_alt_nw(c->precision)};
  double best = INFINITY;
  int bnw = nw0, bS = S0;
  hipEvent_t e0, e1;
  LRIGW_HIP_TRY(hipEventCreate(&e0));
  LRIGW_HIP_TRY(hipEventCreate(&e1));
  const int timing = c->timing;
  c->timing = 0;
  const bool split = ns_chi(c->precision) > 0;
  int bpad = c->chi_pad;
  for (int cand = 0; cand < (split ? 4 : 2); ++cand) {
    const int nw = nws[cand & 1];
    const int pad = (cand >> 1) ? 16 : 8;
    c->chi_nw = nw;
    c->chi_pad = pad;
    int Sp = 1;
    LRIGW_TRY(chi0_plan_splits(c, &Sp));
    std::vector<int> Ss = {std::max(1, Sp / 2), Sp, Sp * 2};
    std::sort(Ss.begin(), Ss.end());
    Ss.erase(std::unique(Ss.begin(), Ss.end()), Ss.end());
    for (int S : Ss) {
      if ((long long)S < chi0_min_splits(c, lrigw_K(c))) continue;
      if ((long long)S > std::max<long long>(1, lrigw_K(c) / 64)) continue;
      c->chi_splits = S;
      // warm-up, then the best of three timed runs
      LRIGW_TRY(run_chi0(c, q, c->d_M, cell.eig, 0, c->d_chi));
      float t = INFINITY;
      for (int rep = 0; rep < 3; ++rep) {
        LRIGW_HIP_TRY(hipEventRecord(e0, s));
        LRIGW_TRY(run_chi0(c, q, c->d_M, cell.eig, 0, c->d_chi));
        LRIGW_HIP_TRY(hipEventRecord(e1, s));
        LRIGW_HIP_TRY(hipEventSynchronize(e1));
        float tr = 0.f;
        LRIGW_HIP_TRY(hipEventElapsedTime(&tr, e0, e1));
        t = std::min(t, tr);
      }
      // a later candidate must be TUNE_MARGIN faster: near-ties resolve to
      // the earliest candidate every time (the K split count changes the
      // order of the FP32 sums, so a stable choice keeps results repeatable)
      if (t < best * (1.0 - TUNE_MARGIN)) {
        best = t;
        bnw = nw;
        bS = S;
        bpad = pad;
      }
    }
  }
  c->chi_nw = bnw;
  c->chi_splits = bS;
  c->chi_pad = bpad;
  *nw_out = bnw;
  *S_out = bS;
  *ms_out = best;
  // split-BF16 Sigma^c kernel variant (timing does not depend on the values)
  if (ns_sig(c->precision) > 0) {
    LRIGW_TRY(run_build_M(c, q, 1, cell.H, cell.evec, c->d_x));
    LRIGW_TRY(zero_fill(s, c->d_wc, (size_t)d.n_freq * d.n_aux * d.n_aux * lrigw_csize(c)));
    double2 *sg = nullptr;
    LRIGW_HIP_TRY(hipMalloc(&sg, (size_t)d.n_k * d.n_qp * d.n_freq * sizeof(double2)));
    double sbest = INFINITY;
    int bvar = c->sig_var;
    for (int var = 0; var < sigma_variants(); ++var) {
      if (!sigma_variant_ok(c, var)) continue;
      c->sig_var = var;
      int rc = run_sigma_c(c, q, c->d_x, c->d_wc, cell.eig, sg);
      float t = INFINITY;
      for (int rep = 0; rep < 3 && rc == LRIGW_OK; ++rep) {
        rc = hipEventRecord(e0, s) == hipSuccess ? LRIGW_OK : LRIGW_ERR_HIP;
        if (rc == LRIGW_OK) rc = run_sigma_c(c, q, c->d_x, c->d_wc, cell.eig, sg);
        if (rc == LRIGW_OK) rc = hipEventRecord(e1, s) == hipSuccess ? LRIGW_OK : LRIGW_ERR_HIP;
        if (rc == LRIGW_OK) rc = hipEventSynchronize(e1) == hipSuccess ? LRIGW_OK : LRIGW_ERR_HIP;
        float tr = 0.f;
        if (rc == LRIGW_OK) rc = hipEventElapsedTime(&tr, e0, e1) == hipSuccess ? LRIGW_OK : LRIGW_ERR_HIP;
        t = std::min(t, tr);
      }
      if (rc != LRIGW_OK) {
        (void)hipFree(sg);
        c->sig_var = bvar;
        return rc;
      }
      if (t < sbest * (1.0 - TUNE_MARGIN)) {
        sbest = t;
        bvar = var;
      }
    }
    (void)hipFree(sg);
    c->sig_var = bvar;
  }
  c->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return LRIGW_OK;
}

static void batch_free(lrigw_batch *b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  for (hipStream_t s : b->cs)
    if (s) hipStreamDestroy(s);
  if (b->fork) hipEventDestroy(b->fork);
  for (hipEvent_t e : b->join)
    if (e) hipEventDestroy(e);
}

static int batch_capture(lrigw_batch *b) {
  const int n = (int)b->cells.size();
  LRIGW_HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = LRIGW_OK;
  hipError_t he = hipEventRecord(b->fork, b->stream);
  for (int i = 0; i < n && rc == LRIGW_OK && he == hipSuccess; ++i) {
    lrigw_batch_cell &cl = b->cells[i];
    lrigw_ctx *c = cl.ctx;
    he = hipStreamWaitEvent(b->cs[i], b->fork, 0);
    if (he != hipSuccess) break;
    b->saved[i] = c->stream;
    c->stream = b->cs[i];
    c->capturing = true;
    const int timing = c->timing;
    c->timing = 0;
    {
      GapScope gap_scope(c);   // checked in lrigw_batch_create; no host round trip under capture
      rc = run_pass(c, cl.H, cl.evec, cl.eig, cl.V, cl.Vcut, cl.p, cl.omega_cell, cl.e_static, cl.n_par, 0, c->d.n_k,
                    cl.sigma, cl.e_qp, cl.z, nullptr);
    }
    c->timing = timing;
    c->capturing = false;
    c->stream = b->saved[i];
    if (rc == LRIGW_OK) he = hipEventRecord(b->join[i], b->cs[i]);
    if (rc == LRIGW_OK && he == hipSuccess) he = hipStreamWaitEvent(b->stream, b->join[i], 0);
  }
  hipGraph_t g = nullptr;
  hipError_t he2 = hipStreamEndCapture(b->stream, &g);
  if (rc != LRIGW_OK) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (he != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return lrigw_hip_error(he, "batch capture", __FILE__, __LINE__);
  }
  if (he2 != hipSuccess) return lrigw_hip_error(he2, "hipStreamEndCapture", __FILE__, __LINE__);
  b->graph = g;
  LRIGW_HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
  return LRIGW_OK;
}

extern "C" {

int lrigw_batch_create(lrigw_batch **out, int n_cells, const lrigw_batch_cell *cells, int autotune, void *hip_stream) {
  (void)hipGetLastError();
  if (!out || n_cells < 1 || n_cells > 64 || !cells) return LRIGW_ERR_ARG;
  if (!hip_stream) return LRIGW_ERR_ARG;   // the legacy default stream cannot be captured
  *out = nullptr;
  for (int i = 0; i < n_cells; ++i) {
    const lrigw_batch_cell &c = cells[i];
    if (!c.ctx || !c.H || !c.evec || !c.eig || !c.V || !c.sigma || !c.e_qp || !c.z) return LRIGW_ERR_ARG;
    if (c.n_par < 1 || c.n_par > 64) return LRIGW_ERR_ARG;
    if (c.p && !(c.omega_cell > 0.0)) return LRIGW_ERR_ARG;
    for (int j = 0; j < i; ++j)
      if (cells[j].ctx == c.ctx) return LRIGW_ERR_ARG;   // one context per cell
  }
  lrigw_batch *b = new (std::nothrow) lrigw_batch();
  if (!b) return LRIGW_ERR_OOM;
  b->cells.assign(cells, cells + n_cells);
  b->stream = (hipStream_t)hip_stream;
  b->cs.assign(n_cells, nullptr);
  b->saved.assign(n_cells, nullptr);
  b->join.assign(n_cells, nullptr);
  b->nw.assign(n_cells, 0);
  b->splits.assign(n_cells, 0);
  b->ms.assign(n_cells, -1.0);
  int rc = LRIGW_OK;
  for (int i = 0; i < n_cells && rc == LRIGW_OK; ++i) {
    lrigw_batch_cell &cl = b->cells[i];
    lrigw_ctx *c = cl.ctx;
    // everything that needs the host happens here, before capture
    if ((rc = driver_buffers(c)) < 0) break;
    if (cl.p && (rc = lrigw_gamma_prepare(c, cl.V, cl.p, cl.omega_cell)) < 0) break;
    if ((rc = chi0_check_gap(c, cl.eig)) < 0) break;
    if (c->sur && (rc = surrogate_prepare(c->sur)) < 0) break;
    if (autotune) {
      GapScope gap_scope(c);
      if ((rc = autotune_chi0(c, cl, &b->nw[i], &b->splits[i], &b->ms[i])) < 0) break;
    } else {
      b->nw[i] = c->chi_nw;
      b->splits[i] = c->chi_splits;
    }
    if (hipStreamCreate(&b->cs[i]) != hipSuccess) rc = LRIGW_ERR_HIP;
    if (rc == LRIGW_OK && hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming) != hipSuccess) rc = LRIGW_ERR_HIP;
  }
  if (rc == LRIGW_OK && hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) rc = LRIGW_ERR_HIP;
  if (rc == LRIGW_OK && hipDeviceSynchronize() != hipSuccess) rc = LRIGW_ERR_HIP;
  if (rc == LRIGW_OK) rc = batch_capture(b);
  if (rc != LRIGW_OK) {
    batch_free(b);
    delete b;
    return rc;
  }
  *out = b;
  return LRIGW_OK;
}

int lrigw_tune(lrigw_ctx *c, const void *H, const void *evec, const double *eig, int *nw, int *splits, int *sigma_variant,
               double *ms) {
  (void)hipGetLastError();
  if (!c || !H || !evec || !eig) return LRIGW_ERR_ARG;
  LRIGW_TRY(driver_buffers(c));
  LRIGW_TRY(chi0_check_gap(c, eig));
  GapScope gap_scope(c);
  lrigw_batch_cell cell = {};
  cell.ctx = c;
  cell.H = H;
  cell.evec = evec;
  cell.eig = eig;
  int a = 0, b = 0;
  double t = 0.0;
  LRIGW_TRY(autotune_chi0(c, cell, &a, &b, &t));
  if (nw) *nw = a;
  if (splits) *splits = b;
  if (sigma_variant) *sigma_variant = c->sig_var;
  if (ms) *ms = t;
  return LRIGW_OK;
}

int lrigw_set_tiles(lrigw_ctx *c, int nw, int splits, int pad, int sigma_variant) {
  if (!c) return LRIGW_ERR_ARG;
  const int dnw = chi0_default_nw(c->precision), anw = chi0_alt_nw(c->precision);
  if (nw != dnw && nw != anw) return LRIGW_ERR_ARG;
  if (pad != 8 && pad != 16) return LRIGW_ERR_ARG;
  if (!sigma_variant_ok(c, sigma_variant)) return LRIGW_ERR_ARG;
  if (splits < 1 || (long long)splits > std::max<long long>(1, lrigw_K(c) / 64) ||
      (long long)splits < chi0_min_splits(c, lrigw_K(c)))
    return LRIGW_ERR_ARG;
  c->chi_nw = nw;
  c->chi_splits = splits;
  c->chi_pad = pad;
  c->sig_var = sigma_variant;
  return LRIGW_OK;
}

int lrigw_get_tiles(const lrigw_ctx *c, int *nw, int *splits, int *pad, int *sigma_variant, int *n_variants) {
  if (!c) return LRIGW_ERR_ARG;
  if (nw) *nw = c->chi_nw;
  if (splits) *splits = c->chi_splits;
  if (pad) *pad = c->chi_pad;
  if (sigma_variant) *sigma_variant = c->sig_var;
  if (n_variants) *n_variants = sigma_variants();
  return LRIGW_OK;
}

int lrigw_batch_run(lrigw_batch *b) {
  (void)hipGetLastError();
  if (!b || !b->exec) return LRIGW_ERR_ARG;
  LRIGW_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  b->launches += 1;
  return LRIGW_OK;
}

int lrigw_batch_status(lrigw_batch *b, int *status) {
  if (!b || !status) return LRIGW_ERR_ARG;
  LRIGW_HIP_TRY(hipStreamSynchronize(b->stream));
  for (size_t i = 0; i < b->cells.size(); ++i) {
    int h[17];
    LRIGW_HIP_TRY(hipMemcpy(h, b->cells[i].ctx->d_info, 17 * sizeof(int), hipMemcpyDeviceToHost));
    status[3 * i + 0] = h[16] == INT_MAX ? -1 : h[16];
    status[3 * i + 1] = h[8];
    status[3 * i + 2] = h[9];
  }
  return LRIGW_OK;
}

int lrigw_batch_tuning(const lrigw_batch *b, int cell, int *nw, int *splits, double *ms) {
  if (!b || cell < 0 || cell >= (int)b->cells.size()) return LRIGW_ERR_ARG;
  if (nw) *nw = b->nw[cell];
  if (splits) *splits = b->splits[cell];
  if (ms) *ms = b->ms[cell];
  return LRIGW_OK;
}

int lrigw_batch_graph_nodes(const lrigw_batch *b, long long *n_nodes) {
  if (!b || !n_nodes || !b->graph) return LRIGW_ERR_ARG;
  size_t n = 0;
  LRIGW_HIP_TRY(hipGraphGetNodes(b->graph, nullptr, &n));
  *n_nodes = (long long)n;
  return LRIGW_OK;
}

int lrigw_batch_destroy(lrigw_batch *b) {
  if (!b) return LRIGW_ERR_ARG;
  if (b->stream) hipStreamSynchronize(b->stream);
  else hipDeviceSynchronize();
  batch_free(b);
  delete b;
  return LRIGW_OK;
}

}  // extern "C"
