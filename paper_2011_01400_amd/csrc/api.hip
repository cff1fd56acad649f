// C interface of the lrigw library: context, validation, driver, timing.
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "lrigw_internal.h"

int lrigw_hip_error(hipError_t e, const char *what, const char *file, int line) {
  if (getenv("LRIGW_VERBOSE")) fprintf(stderr, "lrigw: %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
  return e == hipErrorOutOfMemory ? LRIGW_ERR_OOM : LRIGW_ERR_HIP;
}

int lrigw_launch_check(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return lrigw_hip_error(e, what, __FILE__, __LINE__);
  return LRIGW_OK;
}

size_t lrigw_csize(const lrigw_ctx *c) { return c->precision == LRIGW_FP64 ? sizeof(double2) : sizeof(float2); }
long long lrigw_K(const lrigw_ctx *c) { return (long long)c->d.n_k * c->d.n_occ * c->d.n_unocc; }

// timing mode 2 records only the two MFMA kernel stages (two events per
// launch, nothing between the other kernels of a pass)
static bool stage_timed(const lrigw_ctx *c, const char *name) {
  if (c->timing == 0) return false;
  if (c->timing == 1) return true;
  return std::strcmp(name, "chi0_mfma") == 0 || std::strcmp(name, "sigma_mfma") == 0;
}

void stage_begin(lrigw_ctx *c, const char *name, hipEvent_t *ev) {
  *ev = nullptr;
  if (!stage_timed(c, name)) return;
  if (hipEventCreate(ev) != hipSuccess) { *ev = nullptr; return; }
  hipEventRecord(*ev, c->stream);
}

void stage_end(lrigw_ctx *c, const char *name, hipEvent_t ev) {
  if (!ev || !stage_timed(c, name)) return;
  hipEvent_t e1;
  if (hipEventCreate(&e1) != hipSuccess) return;
  hipEventRecord(e1, c->stream);
  StageTimer &t = c->stages[name];
  t.pending.push_back({ev, e1});
  t.launches += 1;
}

static void free_all(lrigw_ctx *c) {
  void *ptrs[] = {c->d_aux_atom, c->d_basis_off, c->d_aux_off, c->d_kpq, c->d_kmq, c->d_omega, c->d_weight, c->d_wall,
                  c->d_delta, c->d_part, c->d_X, c->d_LV, c->d_s0, c->d_s1, c->d_s2, c->d_s3, c->d_dinv, c->d_info,
                  c->d_bhat, c->d_x1, c->d_M, c->d_x, c->d_chi, c->d_wc, c->d_epsqp, c->d_xs, c->d_ws, c->d_ap, c->d_bt, c->d_chi2, c->d_wc2,
                  c->d_sx, c->d_wmax, c->d_amax, c->d_sitems, c->d_wd, c->d_xo, c->d_sxa, c->d_sxz, c->d_om2,
                  c->d_wsc, c->d_chir, c->d_wr, c->d_Xr, c->d_cdE, c->d_cdS, c->d_cdbad, c->d_sitems_r, c->d_chir2, c->d_wr2, c->d_cut, c->d_bom2, c->d_bcpl, c->d_bwsc, c->d_cf, c->d_grp};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (auto &kv : c->stages)
    for (auto &pr : kv.second.pending) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  for (int i = 0; i < 2; ++i) {
    if (c->ev_chi[i]) hipEventDestroy(c->ev_chi[i]);
    if (c->ev_wc[i]) hipEventDestroy(c->ev_wc[i]);
  }
  if (c->stream2) hipStreamDestroy(c->stream2);
}

// eps_qp[k][n] = eig[k][qp_lo + n]
__global__ void k_qp_bands(const double *__restrict__ eig, int n_k, int n_bands, int qp_lo, int n_qp, double *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_k * n_qp) return;
  out[i] = eig[(long long)(i / n_qp) * n_bands + qp_lo + i % n_qp];
}

__global__ void k_set_int(int *p, int v) { p[threadIdx.x] = v; }

int driver_buffers(lrigw_ctx *c) {
  const Dims &d = c->d;
  size_t cs = lrigw_csize(c);
  if (!c->d_M) LRIGW_HIP_TRY(hipMalloc(&c->d_M, (size_t)lrigw_K(c) * d.n_aux * cs));
  if (!c->d_x) LRIGW_HIP_TRY(hipMalloc(&c->d_x, (size_t)d.n_k * d.n_qp * d.n_bands * d.n_aux * cs));
  if (!c->d_chi) LRIGW_HIP_TRY(hipMalloc(&c->d_chi, (size_t)d.n_freq * d.n_aux * d.n_aux * cs));
  if (!c->d_wc) LRIGW_HIP_TRY(hipMalloc(&c->d_wc, (size_t)d.n_freq * d.n_aux * d.n_aux * cs));
  if (!c->d_epsqp) LRIGW_HIP_TRY(hipMalloc(&c->d_epsqp, (size_t)d.n_k * d.n_qp * sizeof(double)));
  if (!c->d_chi2) LRIGW_HIP_TRY(hipMalloc(&c->d_chi2, (size_t)d.n_freq * d.n_aux * d.n_aux * cs));
  if (!c->d_wc2) LRIGW_HIP_TRY(hipMalloc(&c->d_wc2, (size_t)d.n_freq * d.n_aux * d.n_aux * cs));
  // non-blocking: the context stream may be the legacy default stream, which
  // would otherwise serialize with it (default priority)
  if (!c->stream2) LRIGW_HIP_TRY(hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
  for (int i = 0; i < 2; ++i) {
    if (!c->ev_chi[i]) LRIGW_HIP_TRY(hipEventCreateWithFlags(&c->ev_chi[i], hipEventDisableTiming));
    if (!c->ev_wc[i]) LRIGW_HIP_TRY(hipEventCreateWithFlags(&c->ev_wc[i], hipEventDisableTiming));
  }
  return LRIGW_OK;
}

// One pass over q_first..q_last-1 (and the QP step when every q was done).
// Software pipeline over q on two streams: `stream` builds M and the response
// of q (into one of two chi buffers) and then the Sigma^c contribution of q-1;
// `stream2` screens q (into one of two W^c buffers) as soon as its response is
// ready, so the latency-bound screening overlaps the MFMA-bound response of
// q+1.  Events order the buffer reuse:
//   chi[q&1] is rewritten only after sigma(q-2), which waited for screen(q-2);
//   W[q&1] is rewritten by screen(q), which starts after chi0(q), issued after
//   sigma(q-2) on `stream`.
// The screening status is folded on the device (d_info[16] = first failing q)
// and read once at the end (not under graph capture).  With a surrogate
// attached (its per-q work shares the screening workspaces), and under graph
// capture (the batched form overlaps whole cells on streams of their own
// instead), the pass runs on `stream` alone.
// q per screening group: as many as fit 8 GiB of responses, W^c and FP64
// workspace (at most 8); 1 (no grouping) when one q alone exceeds that
static int pass_group_size(const lrigw_ctx *c, int nq) {
  const Dims &d = c->d;
  const size_t per_q = 4 * (size_t)d.n_freq * d.n_aux * d.n_aux * lrigw_csize(c) +
                       (size_t)group_ws_elems(c, 1) * sizeof(double2);
  const size_t fit = ((size_t)8 << 30) / per_q;
  return (int)std::max<size_t>(1, std::min<size_t>({fit, (size_t)8, (size_t)nq}));
}

// two sets of G response and G W^c blocks (one group is screened while the
// next one's responses are built), and the screening workspace of G q
static int group_buffers(lrigw_ctx *c, int G) {
  const Dims &d = c->d;
  const size_t need = 4 * (size_t)G * d.n_freq * d.n_aux * d.n_aux * lrigw_csize(c) +
                      (size_t)group_ws_elems(c, G) * sizeof(double2);
  if (need > c->grp_bytes) {
    if (c->d_grp) LRIGW_HIP_TRY(hipFree(c->d_grp));
    c->d_grp = nullptr;
    c->grp_bytes = 0;
    LRIGW_HIP_TRY(hipMalloc(&c->d_grp, need));
    c->grp_bytes = need;
  }
  c->grp_cap = G;
  return LRIGW_OK;
}

// The end of a pass: the screening status (not under capture), then the QP
// step when every q was done.
static int pass_finish(lrigw_ctx *c, const double *eig, const double *e_static, int n_par, bool all_q, void *sigma,
                       double *e_qp, double *z, int *info) {
  const Dims &d = c->d;
  const hipStream_t s = c->stream;
  if (!c->capturing) {
    int h = INT_MAX;
    LRIGW_HIP_TRY(hipMemcpyAsync(&h, c->d_info + 16, sizeof(int), hipMemcpyDeviceToHost, s));
    LRIGW_HIP_TRY(hipStreamSynchronize(s));
    if (h != INT_MAX) {
      if (info) *info = h;
      return LRIGW_ERR_NOT_HPD;
    }
  }
  if (!all_q) return LRIGW_OK;
  const int nkq = d.n_k * d.n_qp;
  hipLaunchKernelGGL(k_qp_bands, dim3((nkq + 255) / 256), dim3(256), 0, s, eig, d.n_k, d.n_bands, d.qp_lo, d.n_qp,
                     c->d_epsqp);
  LRIGW_TRY(lrigw_launch_check("qp_bands"));
  int qinfo = 0;
  const int rc = lrigw_qp(c, sigma, c->d_epsqp, e_static, n_par, e_qp, z, &qinfo);
  if (info) *info = qinfo;
  return rc;
}

int run_pass(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
             const void *p, double omega_cell, const double *e_static, int n_par, int q_first, int q_last, void *sigma,
             double *e_qp, double *z, int *info) {
  (void)omega_cell;
  const Dims &d = c->d;
  if (c->gap_trusted == 0) LRIGW_TRY(chi0_check_gap(c, eig));
  GapScope gap_scope(c);
  const bool all_q = (q_first == 0 && q_last == d.n_k);
  const hipStream_t s = c->stream;
  const bool overlap = (c->sur == nullptr) && !c->capturing;
  const hipStream_t s2 = overlap ? c->stream2 : s;
  LRIGW_TRY(zero_fill(s, sigma, (size_t)d.n_k * d.n_qp * d.n_freq * sizeof(double2)));
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->d_info + 16, INT_MAX);
  // V(q) (and V^cut) factors of every q at once (not under graph capture)
  CoulombScope coulomb_scope(c);
  if (!c->capturing) LRIGW_TRY(coulomb_factors(c, V, Vcut, q_first, q_last));
  const size_t vstride = (size_t)d.n_aux * d.n_aux;
  // two buffers in either mode: Sigma^c(q-1) is issued after screen(q)
  void *chi[2] = {c->d_chi, c->d_chi2};
  void *wc[2] = {c->d_wc, c->d_wc2};
  const bool was_capturing = c->capturing;
  // Grouped form (not under capture, no surrogate, no direction average): the
  // q are taken in groups of G, and one screening covers a group's G N_w
  // planes (wide launches instead of N_q chains of small latency-bound ones).
  // Per group g, on `stream`: M and the response of each q of g, then x and
  // Sigma^c of each q of g - 1 (after its screening); the screening of g runs
  // on stream2 after that self-energy, beside the responses of g + 1, so no
  // screening runs beside the self-energy kernel.  Buffer sets alternate by
  // group: a response set is rewritten only after the self-energy of its
  // group, which waited for the screening that read it; a W^c set is
  // rewritten by a screening that starts after the self-energy that read it.
  const int G = (!was_capturing && c->sur == nullptr && c->n_gdir == 0) ? pass_group_size(c, q_last - q_first) : 1;
  if (G > 1) {
    LRIGW_TRY(group_buffers(c, G));
    const size_t cs = lrigw_csize(c), blk = (size_t)d.n_freq * vstride * cs;
    char *gchi[2] = {(char *)c->d_grp, (char *)c->d_grp + G * blk};
    char *gwc[2] = {(char *)c->d_grp + 2 * G * blk, (char *)c->d_grp + 3 * G * blk};
    double2 *gws = (double2 *)((char *)c->d_grp + 4 * G * blk);
    c->capturing = true;   // device-side status
    int rc = LRIGW_OK;
    const int ng = (q_last - q_first + G - 1) / G;
    for (int g = 0; g <= ng && rc == LRIGW_OK; ++g) {
      const int q0 = q_first + g * G, nq = g < ng ? std::min(G, q_last - q0) : 0;
      for (int j = 0; j < nq && rc == LRIGW_OK; ++j) {
        const int q = q0 + j;
        if ((rc = lrigw_build_M(c, q, 0, H, evec, c->d_M)) < 0) break;
        rc = lrigw_chi0(c, q, c->d_M, eig, (p && q == 0) ? 1 : 0, gchi[g & 1] + j * blk);
      }
      if (rc < 0) break;
      if (g > 0) {
        // Sigma^c of the previous group, after its screening
        const int pg = g - 1, p0 = q_first + pg * G, pn = std::min(G, q_last - p0);
        if (hipStreamWaitEvent(s, c->ev_wc[pg & 1], 0) != hipSuccess) {
          rc = LRIGW_ERR_HIP;
          break;
        }
        for (int j = 0; j < pn && rc == LRIGW_OK; ++j) {
          const int q = p0 + j;
          if ((rc = lrigw_build_M(c, q, 1, H, evec, c->d_x)) < 0) break;
          rc = lrigw_sigma_c(c, q, c->d_x, gwc[pg & 1] + j * blk, eig, sigma);
        }
        if (rc < 0) break;
      }
      if (nq == 0) break;
      // the screening of this group on stream2, after everything issued so far
      if (hipEventRecord(c->ev_chi[g & 1], s) != hipSuccess || hipStreamWaitEvent(s2, c->ev_chi[g & 1], 0) != hipSuccess) {
        rc = LRIGW_ERR_HIP;
        break;
      }
      c->stream = s2;
      hipEvent_t ev;
      stage_begin(c, "screen", &ev);
      if (Vcut && q0 == 0) {
        // V[0] is V^cut(0): q = 0 alone, then the rest of the group
        rc = run_screen_group(c, 0, 1, gchi[g & 1], V, nullptr, gwc[g & 1], gws);
        if (rc == LRIGW_OK && nq > 1)
          rc = run_screen_group(c, 1, nq - 1, gchi[g & 1] + blk, (const double2 *)V + vstride,
                                (const double2 *)Vcut + vstride, gwc[g & 1] + blk, gws);
      } else {
        const void *Vcg = Vcut ? (const void *)((const double2 *)Vcut + q0 * vstride) : nullptr;
        rc = run_screen_group(c, q0, nq, gchi[g & 1], (const double2 *)V + q0 * vstride, Vcg, gwc[g & 1], gws);
      }
      stage_end(c, "screen", ev);
      if (rc == LRIGW_OK && hipEventRecord(c->ev_wc[g & 1], s2) != hipSuccess) rc = LRIGW_ERR_HIP;
      c->stream = s;
    }
    c->stream = s;
    c->capturing = was_capturing;
    if (rc < 0) return rc;
    return pass_finish(c, eig, e_static, n_par, all_q, sigma, e_qp, z, info);
  }
  c->capturing = true;   // screening: device-side status, no host round trip
  int rc = LRIGW_OK;
  for (int q = q_first; q <= q_last && rc == LRIGW_OK; ++q) {
    if (q < q_last) {
      const int b = q & 1;
      if ((rc = lrigw_build_M(c, q, 0, H, evec, c->d_M)) < 0) break;
      const int g = (p && q == 0) ? 1 : 0;
      if (g && c->n_gdir > 0) {
        // W^c(0) averaged over the directions, on `stream` (exact response;
        // the other buffer, first used by q = 1, is the scratch)
        if ((rc = run_gamma_average(c, eig, V, false, chi[b], wc[1 - b], wc[b])) < 0) break;
        if (overlap && hipEventRecord(c->ev_wc[b], s) != hipSuccess) {
          rc = LRIGW_ERR_HIP;
          break;
        }
      } else {
      if (c->sur) rc = lrigw_chi0_surrogate(c, c->sur, q, c->d_M, eig, g, c->sur_threshold, chi[b]);
      else rc = lrigw_chi0(c, q, c->d_M, eig, g, chi[b]);
      if (rc < 0) break;
      if (overlap) {
        if (hipEventRecord(c->ev_chi[b], s) != hipSuccess || hipStreamWaitEvent(s2, c->ev_chi[b], 0) != hipSuccess) {
          rc = LRIGW_ERR_HIP;
          break;
        }
      }
      c->stream = s2;
      // V^cut(q) in the numerator for q != 0; V[0] already is V^cut(0)
      const void *Vcq = (Vcut && q > 0) ? (const void *)((const double2 *)Vcut + q * vstride) : nullptr;
      rc = lrigw_screen(c, q, chi[b], (const double2 *)V + q * vstride, Vcq, wc[b], nullptr);
      c->stream = s;
      if (rc < 0) break;
      if (overlap && hipEventRecord(c->ev_wc[b], s2) != hipSuccess) {
        rc = LRIGW_ERR_HIP;
        break;
      }
      }
    }
    if (q > q_first) {
      const int pq = q - 1, b = pq & 1;
      if ((rc = lrigw_build_M(c, pq, 1, H, evec, c->d_x)) < 0) break;
      if (overlap && hipStreamWaitEvent(s, c->ev_wc[b], 0) != hipSuccess) {
        rc = LRIGW_ERR_HIP;
        break;
      }
      if ((rc = lrigw_sigma_c(c, pq, c->d_x, wc[b], eig, sigma)) < 0) break;
    }
  }
  c->stream = s;
  c->capturing = was_capturing;
  if (rc < 0) return rc;
  return pass_finish(c, eig, e_static, n_par, all_q, sigma, e_qp, z, info);
}

// Sigma^c at real energies over every q by contour deformation: per q the
// response and W^c on the imaginary grid and on the real grid, the pairs of
// the QP bands, and the combination at the n_e energy sets.  As in run_pass,
// `stream2` screens q (both plane sets, into one of two buffer pairs) while
// the responses of q+1 are built on `stream`; the same events order the
// buffer reuse, and the screening status is folded on the device.  The
// exact response is used (an attached surrogate is not).
int run_cd_pass(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                const void *p, double omega_cell, int n_e, const double *E, double *sigma_e, int *n_bad) {
  const Dims &d = c->d;
  LRIGW_TRY(driver_buffers(c));
  if (p) LRIGW_TRY(lrigw_gamma_prepare(c, V, p, omega_cell));
  LRIGW_TRY(chi0_check_gap(c, eig));
  GapScope gap_scope(c);
  const hipStream_t s = c->stream, s2 = c->stream2;
  LRIGW_TRY(zero_fill(s, sigma_e, (size_t)n_e * d.n_k * d.n_qp * sizeof(double)));
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, c->d_info + 16, INT_MAX);
  CoulombScope coulomb_scope(c);
  if (!c->capturing) LRIGW_TRY(coulomb_factors(c, V, Vcut, 0, d.n_k));
  const size_t vstride = (size_t)d.n_aux * d.n_aux;
  void *chi[2] = {c->d_chi, c->d_chi2}, *wc[2] = {c->d_wc, c->d_wc2};
  void *chir[2] = {c->d_chir, c->d_chir2}, *wr[2] = {c->d_wr, c->d_wr2};
  c->capturing = true;   // screening: device-side status, no host round trip
  int rc = LRIGW_OK;
  for (int q = 0; q <= d.n_k && rc == LRIGW_OK; ++q) {
    if (q < d.n_k) {
      const int b = q & 1, g = (p && q == 0) ? 1 : 0;
      const double2 *Vq = (const double2 *)V + q * vstride;
      if ((rc = lrigw_build_M(c, q, 0, H, evec, c->d_M)) < 0) break;
      if (g && c->n_gdir > 0) {
        // both plane sets of W^c(0) averaged over the directions, on `stream`
        if ((rc = run_gamma_average(c, eig, Vq, false, chi[b], wc[1 - b], wc[b])) < 0) break;
        if ((rc = run_gamma_average(c, eig, Vq, true, chir[b], wr[1 - b], wr[b])) < 0) break;
        if (hipEventRecord(c->ev_wc[b], s) != hipSuccess) {
          rc = LRIGW_ERR_HIP;
          break;
        }
        continue;
      }
      if ((rc = run_chi0(c, q, c->d_M, eig, g, chi[b])) < 0) break;
      if ((rc = run_chi0_real(c, q, c->d_M, eig, g, chir[b])) < 0) break;
      if (hipEventRecord(c->ev_chi[b], s) != hipSuccess || hipStreamWaitEvent(s2, c->ev_chi[b], 0) != hipSuccess) {
        rc = LRIGW_ERR_HIP;
        break;
      }
      c->stream = s2;
      const void *Vcq = (Vcut && q > 0) ? (const void *)((const double2 *)Vcut + q * vstride) : nullptr;
      rc = run_screen(c, q, chi[b], Vq, Vcq, wc[b], nullptr);
      if (rc == LRIGW_OK) rc = run_screen_n(c, q, chir[b], Vq, Vcq, wr[b], nullptr, c->n_real);
      c->stream = s;
      if (rc < 0) break;
      if (hipEventRecord(c->ev_wc[b], s2) != hipSuccess) {
        rc = LRIGW_ERR_HIP;
        break;
      }
    }
    if (q > 0) {
      const int pq = q - 1, b = pq & 1;
      if ((rc = lrigw_build_M(c, pq, 1, H, evec, c->d_x)) < 0) break;
      if (hipStreamWaitEvent(s, c->ev_wc[b], 0) != hipSuccess) {
        rc = LRIGW_ERR_HIP;
        break;
      }
      rc = run_sigma_cd(c, pq, c->d_x, wc[b], wr[b], eig, n_e, E, sigma_e);
    }
  }
  c->stream = s;
  c->capturing = false;
  if (rc < 0) return rc;
  int h = INT_MAX;
  LRIGW_HIP_TRY(hipMemcpyAsync(&h, c->d_info + 16, sizeof(int), hipMemcpyDeviceToHost, s));
  LRIGW_HIP_TRY(hipStreamSynchronize(s));
  if (h != INT_MAX) return LRIGW_ERR_NOT_HPD;
  int bad = 0;
  LRIGW_TRY(cd_count_nan(c, sigma_e, n_e * d.n_k * d.n_qp, &bad));
  if (n_bad) *n_bad = bad;
  return bad ? LRIGW_WARN_CD_RANGE : LRIGW_OK;
}

extern "C" {

const char *lrigw_strerror(int code) {
  switch (code) {
    case LRIGW_OK: return "ok";
    case LRIGW_ERR_ARG: return "invalid argument";
    case LRIGW_ERR_OOM: return "device out of memory";
    case LRIGW_ERR_HIP: return "HIP runtime error";
    case LRIGW_ERR_NOT_HPD: return "matrix not Hermitian positive definite";
    case LRIGW_ERR_NOCONV: return "iteration did not converge";
    case LRIGW_WARN_QP_NOCONV: return "warning: some quasiparticle equations had no root";
    case LRIGW_WARN_PADE_TRUNC: return "warning: some Pade fits were truncated";
    case LRIGW_WARN_CD_RANGE: return "warning: some residue frequencies lie beyond the real grid (NaN returned)";
    default: return "unknown status";
  }
}

int lrigw_create(lrigw_ctx **out, const lrigw_system *sys, int precision, void *hip_stream) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!out || !sys || !sys->basis_off || !sys->aux_off) return LRIGW_ERR_ARG;
  *out = nullptr;
  if (precision < LRIGW_FP64 || precision > LRIGW_SPLIT_F16) return LRIGW_ERR_ARG;
  if (sys->n_atoms < 1 || sys->nk[0] < 1 || sys->nk[1] < 1 || sys->nk[2] < 1) return LRIGW_ERR_ARG;
  if (sys->basis_off[0] != 0 || sys->aux_off[0] != 0) return LRIGW_ERR_ARG;
  int nb_max = 0;
  for (int a = 0; a < sys->n_atoms; ++a) {
    int nb = sys->basis_off[a + 1] - sys->basis_off[a];
    int na = sys->aux_off[a + 1] - sys->aux_off[a];
    if (nb < 1 || na < 1) return LRIGW_ERR_ARG;
    if (nb > nb_max) nb_max = nb;
  }
  int n_b = sys->basis_off[sys->n_atoms];
  int n_aux = sys->aux_off[sys->n_atoms];
  if (sys->n_bands < 2 || sys->n_bands > n_b) return LRIGW_ERR_ARG;
  if (sys->n_occ < 1 || sys->n_occ >= sys->n_bands || sys->n_occ > 64) return LRIGW_ERR_ARG;
  if (sys->n_freq < 1 || sys->n_freq > 4096 || !(sys->x0 > 0.0)) return LRIGW_ERR_ARG;
  if (sys->qp_lo < 0 || sys->n_qp < 1 || sys->n_qp > 64 || sys->qp_lo + sys->n_qp > sys->n_bands) return LRIGW_ERR_ARG;
  long long n_k = (long long)sys->nk[0] * sys->nk[1] * sys->nk[2];
  if (n_k > 65535) return LRIGW_ERR_ARG;

  lrigw_ctx *c = new (std::nothrow) lrigw_ctx();
  if (!c) return LRIGW_ERR_OOM;
  Dims &d = c->d;
  d.n_atoms = sys->n_atoms;
  for (int i = 0; i < 3; ++i) d.nk[i] = sys->nk[i];
  d.n_k = (int)n_k;
  d.n_b = n_b;
  d.n_aux = n_aux;
  d.n_bands = sys->n_bands;
  d.n_occ = sys->n_occ;
  d.n_unocc = sys->n_bands - sys->n_occ;
  d.n_freq = sys->n_freq;
  d.x0 = sys->x0;
  d.mu = sys->mu;
  d.qp_lo = sys->qp_lo;
  d.n_qp = sys->n_qp;
  d.nb_max = nb_max;
  c->precision = precision;
  c->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return LRIGW_ERR_HIP;
  }
  c->basis_off.assign(sys->basis_off, sys->basis_off + d.n_atoms + 1);
  c->aux_off.assign(sys->aux_off, sys->aux_off + d.n_atoms + 1);

  int rc = run_grids(c);
  // device address of the allocation-free fit's fixed workspace, once per device
  if (rc >= 0) rc = fit_scratch_prepare(c->device);
  if (rc < 0) {
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return LRIGW_OK;
}

int lrigw_destroy(lrigw_ctx *c) {
  if (!c) return LRIGW_ERR_ARG;
  if (c->stream) hipStreamSynchronize(c->stream);
  else hipDeviceSynchronize();
  if (c->stream2) hipStreamSynchronize(c->stream2);
  free_all(c);
  delete c;
  return LRIGW_OK;
}

int lrigw_get_sizes(const lrigw_ctx *c, lrigw_sizes *o) {
  if (!c || !o) return LRIGW_ERR_ARG;
  const Dims &d = c->d;
  o->n_k = d.n_k;
  o->n_b = d.n_b;
  o->n_aux = d.n_aux;
  o->n_bands = d.n_bands;
  o->n_freq = d.n_freq;
  o->nb_max = d.nb_max;
  o->h_elems = (long long)d.n_k * d.nb_max * d.n_bands * d.n_aux;
  o->m_chi_elems = lrigw_K(c) * d.n_aux;
  o->m_sig_elems = (long long)d.n_k * d.n_qp * d.n_bands * d.n_aux;
  o->m_x_elems = (long long)d.n_k * d.n_qp * d.n_occ * d.n_aux;
  o->w_elems = (long long)d.n_freq * d.n_aux * d.n_aux;
  o->sigma_elems = (long long)d.n_k * d.n_qp * d.n_freq;
  return LRIGW_OK;
}

int lrigw_grids(lrigw_ctx *c, double *omega, double *weight, int *kpq, int *kmq) {
  if (!c) return LRIGW_ERR_ARG;
  const Dims &d = c->d;
  size_t kk = (size_t)d.n_k * d.n_k * sizeof(int);
  if (omega) LRIGW_HIP_TRY(hipMemcpyAsync(omega, c->d_omega, d.n_freq * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (weight) LRIGW_HIP_TRY(hipMemcpyAsync(weight, c->d_weight, d.n_freq * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (kpq) LRIGW_HIP_TRY(hipMemcpyAsync(kpq, c->d_kpq, kk, hipMemcpyDeviceToDevice, c->stream));
  if (kmq) LRIGW_HIP_TRY(hipMemcpyAsync(kmq, c->d_kmq, kk, hipMemcpyDeviceToDevice, c->stream));
  return LRIGW_OK;
}

int lrigw_lri_ft(lrigw_ctx *c, const double *lri_R, const int *R_list, int nR, const void *evec, void *H_out) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!c || !lri_R || !R_list || nR < 1 || !evec || !H_out) return LRIGW_ERR_ARG;
  hipEvent_t ev;
  stage_begin(c, "lri_ft", &ev);
  int rc = run_lri_ft(c, lri_R, R_list, nR, evec, H_out);
  stage_end(c, "lri_ft", ev);
  return rc;
}

int lrigw_build_M(lrigw_ctx *c, int iq, int slice, const void *H, const void *evec, void *M_out) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!c || !H || !evec || !M_out) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k || slice < 0 || slice > 2) return LRIGW_ERR_ARG;
  hipEvent_t ev;
  stage_begin(c, "build_M", &ev);
  int rc = run_build_M(c, iq, slice, H, evec, M_out);
  stage_end(c, "build_M", ev);
  return rc;
}

int lrigw_chi0(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!c || !M || !eig || !chi_out) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k) return LRIGW_ERR_ARG;
  if (apply_gamma && (iq != 0 || !c->gamma_ready)) return LRIGW_ERR_ARG;
  return run_chi0(c, iq, M, eig, apply_gamma, chi_out);
}

int lrigw_chi0_surrogate(lrigw_ctx *c, lrigw_surrogate *sg, int iq, const void *M, const double *eig, int apply_gamma,
                         double threshold, void *chi_out) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!c || !sg || !M || !eig || !chi_out || !(threshold >= 0.0)) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k) return LRIGW_ERR_ARG;
  if (apply_gamma && (iq != 0 || !c->gamma_ready)) return LRIGW_ERR_ARG;
  return run_chi0_surrogate(c, sg, iq, M, eig, apply_gamma, threshold, chi_out);
}

int lrigw_set_surrogate(lrigw_ctx *c, lrigw_surrogate *sg, double threshold) {
  if (!c || (sg && !(threshold >= 0.0))) return LRIGW_ERR_ARG;
  c->sur = sg;
  c->sur_threshold = threshold;
  return LRIGW_OK;
}

int lrigw_gamma_prepare(lrigw_ctx *c, const void *Vcut0, const void *p, double omega_cell) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!c || !Vcut0 || !p || !(omega_cell > 0.0)) return LRIGW_ERR_ARG;
  return run_gamma_prepare(c, Vcut0, p, omega_cell);
}

int lrigw_set_gamma_directions(lrigw_ctx *c, int n_dir, const void *p_dirs, const double *weights) {
  if (!c || n_dir < 0 || n_dir > 64) return LRIGW_ERR_ARG;
  if (n_dir == 0) {
    c->n_gdir = 0;
    c->gdir_p = nullptr;
    c->gdir_w.clear();
    return LRIGW_OK;
  }
  if (!p_dirs || !weights) return LRIGW_ERR_ARG;
  for (int i = 0; i < n_dir; ++i)
    if (!std::isfinite(weights[i])) return LRIGW_ERR_ARG;
  c->gdir_w.assign(weights, weights + n_dir);
  c->gdir_p = p_dirs;
  c->n_gdir = n_dir;
  return LRIGW_OK;
}

int lrigw_screen(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!c || !chi || !V || !Wc_out) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k) return LRIGW_ERR_ARG;
  hipEvent_t ev;
  stage_begin(c, "screen", &ev);
  int rc = run_screen(c, iq, chi, V, Vcut, Wc_out, info);
  stage_end(c, "screen", ev);
  return rc;
}

int lrigw_sigma_c(lrigw_ctx *c, int iq, const void *x, const void *Wc, const double *eig, void *sigma_acc) {
  (void)hipGetLastError();  // drop a stale error another library left behind
  if (!c || !x || !Wc || !eig || !sigma_acc) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k) return LRIGW_ERR_ARG;
  return run_sigma_c(c, iq, x, Wc, eig, sigma_acc);
}

int lrigw_sigma_x(lrigw_ctx *c, int iq, const void *xo, const void *V, double *sigma_x) {
  (void)hipGetLastError();
  if (!c || !xo || !V || !sigma_x) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k) return LRIGW_ERR_ARG;
  return run_sigma_x(c, iq, xo, V, sigma_x);
}

int lrigw_sigma_x_pass(lrigw_ctx *c, const void *H, const void *evec, const void *V, double *sigma_x) {
  (void)hipGetLastError();
  if (!c || !H || !evec || !V || !sigma_x) return LRIGW_ERR_ARG;
  const Dims &d = c->d;
  if (!c->d_xo) LRIGW_HIP_TRY(hipMalloc(&c->d_xo, (size_t)d.n_k * d.n_qp * d.n_occ * d.n_aux * lrigw_csize(c)));
  LRIGW_TRY(zero_fill(c->stream, sigma_x, (size_t)d.n_k * d.n_qp * sizeof(double)));
  const size_t vstride = (size_t)d.n_aux * d.n_aux;
  for (int q = 0; q < d.n_k; ++q) {
    LRIGW_TRY(run_build_M(c, q, 2, H, evec, c->d_xo));
    LRIGW_TRY(run_sigma_x(c, q, c->d_xo, (const double2 *)V + q * vstride, sigma_x));
  }
  return LRIGW_OK;
}

int lrigw_lri_fit(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T, double scale,
                  double *C, int *info) {
  (void)hipGetLastError();
  if (info) *info = -1;
  if (!c || !V || !T || !C) return LRIGW_ERR_ARG;
  if (batch < 1 || batch > 65535 || n < 1 || n_keep < 1 || n_keep > n || nrhs < 1) return LRIGW_ERR_ARG;
  return run_lri_fit(c, batch, n, n_keep, nrhs, V, T, scale, C, info);
}

int lrigw_lri_fit_noalloc(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T,
                          double scale, double *C, int *info) {
  (void)hipGetLastError();
  if (info) *info = -1;
  if (!c || !V || !T || !C) return LRIGW_ERR_ARG;
  if (batch < 1 || batch > 65535 || n < 1 || n_keep < 1 || n_keep > n || nrhs < 1) return LRIGW_ERR_ARG;
  return run_lri_fit_noalloc(c, batch, n, n_keep, nrhs, V, T, scale, C, info);
}

int lrigw_qp(lrigw_ctx *c, const void *sigma, const double *eps_qp, const double *e_static, int n_par, double *e_qp,
             double *z, int *info) {
  (void)hipGetLastError();
  if (!c || !sigma || !eps_qp || !e_qp || !z) return LRIGW_ERR_ARG;
  if (n_par < 1 || n_par > 64) return LRIGW_ERR_ARG;
  hipEvent_t ev;
  stage_begin(c, "qp", &ev);
  int rc = run_qp(c, sigma, eps_qp, e_static, n_par, e_qp, z, info);
  stage_end(c, "qp", ev);
  return rc;
}

int lrigw_set_real_grid(lrigw_ctx *c, int n_r, double omega_max, double eta) {
  (void)hipGetLastError();
  if (!c) return LRIGW_ERR_ARG;
  return run_set_real_grid(c, n_r, omega_max, eta);
}

int lrigw_chi0_real(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out) {
  (void)hipGetLastError();
  if (!c || !M || !eig || !chi_out) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k) return LRIGW_ERR_ARG;
  if (apply_gamma && (iq != 0 || !c->gamma_ready)) return LRIGW_ERR_ARG;
  if (c->real_eta > 0.0) return LRIGW_ERR_ARG;   // the broadened grid is for the passes only
  hipEvent_t ev;
  stage_begin(c, "chi0_real", &ev);
  int rc = run_chi0_real(c, iq, M, eig, apply_gamma, chi_out);
  stage_end(c, "chi0_real", ev);
  return rc;
}

int lrigw_screen_real(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info) {
  (void)hipGetLastError();
  if (!c || !chi || !V || !Wc_out) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k || c->n_real < 4 || c->real_eta > 0.0) return LRIGW_ERR_ARG;
  hipEvent_t ev;
  stage_begin(c, "screen_real", &ev);
  int rc = run_screen_n(c, iq, chi, V, Vcut, Wc_out, info, c->n_real);
  stage_end(c, "screen_real", ev);
  return rc;
}

int lrigw_sigma_cd(lrigw_ctx *c, int iq, const void *x, const void *Wc, const void *Wr, const double *eig, int n_e,
                   const double *E, double *sigma_e) {
  (void)hipGetLastError();
  if (!c || !x || !Wc || !Wr || !eig || !E || !sigma_e) return LRIGW_ERR_ARG;
  if (iq < 0 || iq >= c->d.n_k || c->real_eta > 0.0) return LRIGW_ERR_ARG;
  return run_sigma_cd(c, iq, x, Wc, Wr, eig, n_e, E, sigma_e);
}

int lrigw_sigma_cd_pass(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                        const void *p, double omega_cell, int n_e, const double *E, double *sigma_e, int *n_bad) {
  (void)hipGetLastError();
  if (n_bad) *n_bad = 0;
  if (!c || !H || !evec || !eig || !V || !E || !sigma_e) return LRIGW_ERR_ARG;
  if (c->n_real < 4 || n_e < 1 || n_e > 4 || c->capturing) return LRIGW_ERR_ARG;
  if (p && !(omega_cell > 0.0)) return LRIGW_ERR_ARG;
  if (c->real_eta > 0.0) return run_cd_pass_broadened(c, H, evec, eig, V, Vcut, p, omega_cell, n_e, E, sigma_e, n_bad);
  return run_cd_pass(c, H, evec, eig, V, Vcut, p, omega_cell, n_e, E, sigma_e, n_bad);
}

int lrigw_g0w0_cd(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                  const void *p, double omega_cell, const double *e_static, double delta, double *sigma3, double *e_qp,
                  double *z, int *n_bad) {
  (void)hipGetLastError();
  if (n_bad) *n_bad = 0;
  if (!c || !H || !evec || !eig || !V || !e_qp || !z) return LRIGW_ERR_ARG;
  if (c->n_real < 4 || !(delta > 0.0) || !std::isfinite(delta) || c->capturing) return LRIGW_ERR_ARG;
  if (p && !(omega_cell > 0.0)) return LRIGW_ERR_ARG;
  double *S = sigma3 ? sigma3 : c->d_cdS;
  LRIGW_TRY(cd_energies(c, eig, delta));
  const int rc = c->real_eta > 0.0
                     ? run_cd_pass_broadened(c, H, evec, eig, V, Vcut, p, omega_cell, 3, c->d_cdE, S, n_bad)
                     : run_cd_pass(c, H, evec, eig, V, Vcut, p, omega_cell, 3, c->d_cdE, S, n_bad);
  if (rc < 0) return rc;
  LRIGW_TRY(cd_qp_linear(c, S, e_static, delta, e_qp, z));
  return rc;
}

int lrigw_qp_cd(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                const void *p, double omega_cell, const double *e_static, double delta, int n_iter, int warm,
                double *sigma3, double *e_qp, double *z, int *n_bad) {
  (void)hipGetLastError();
  if (n_bad) *n_bad = 0;
  if (!c || !H || !evec || !eig || !V || !e_qp || !z) return LRIGW_ERR_ARG;
  if (c->n_real < 4 || !(delta > 0.0) || !std::isfinite(delta) || c->capturing || n_iter < 1 || n_iter > 64 ||
      warm < 0 || warm > 1)
    return LRIGW_ERR_ARG;
  if (p && !(omega_cell > 0.0)) return LRIGW_ERR_ARG;
  double *S = sigma3 ? sigma3 : c->d_cdS;
  int rc = LRIGW_OK;
  for (int it = 0; it < n_iter; ++it) {
    // energies E - delta, E, E + delta of the current iterate (E_0 = e_n)
    LRIGW_TRY(cd_newton(c, eig, nullptr, nullptr, delta, e_qp, nullptr, it == 0 && !warm));
    rc = c->real_eta > 0.0 ? run_cd_pass_broadened(c, H, evec, eig, V, Vcut, p, omega_cell, 3, c->d_cdE, S, n_bad)
                           : run_cd_pass(c, H, evec, eig, V, Vcut, p, omega_cell, 3, c->d_cdE, S, n_bad);
    if (rc < 0) return rc;
    LRIGW_TRY(cd_newton(c, eig, S, e_static, delta, e_qp, z, 0));
  }
  return rc;
}

int lrigw_pade_eval(lrigw_ctx *c, const void *sigma, int n_par, int n_e, const double *E, void *out) {
  (void)hipGetLastError();
  if (!c || !sigma || !E || !out || n_par < 1 || n_par > 64 || n_e < 1) return LRIGW_ERR_ARG;
  return run_pade_eval(c, sigma, n_par, n_e, E, out);
}

int lrigw_g0w0(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
               const void *p, double omega_cell, const double *e_static, int n_par, int q_first, int q_last, void *sigma,
               double *e_qp, double *z, int *info) {
  (void)hipGetLastError();
  if (!c || !H || !evec || !eig || !V || !sigma) return LRIGW_ERR_ARG;
  const Dims &d = c->d;
  if (q_first < 0 || q_last > d.n_k || q_first >= q_last) return LRIGW_ERR_ARG;
  bool all_q = (q_first == 0 && q_last == d.n_k);
  if (all_q && (!e_qp || !z)) return LRIGW_ERR_ARG;
  if (n_par < 1 || n_par > 64) return LRIGW_ERR_ARG;
  LRIGW_TRY(driver_buffers(c));
  if (p && q_first == 0) LRIGW_TRY(lrigw_gamma_prepare(c, V, p, omega_cell));
  return run_pass(c, H, evec, eig, V, Vcut, p, omega_cell, e_static, n_par, q_first, q_last, sigma, e_qp, z, info);
}

int lrigw_set_timing(lrigw_ctx *c, int on) {
  if (!c) return LRIGW_ERR_ARG;
  if (on < 0 || on > 2) return LRIGW_ERR_ARG;
  c->timing = on;
  return LRIGW_OK;
}

double lrigw_stage_ms(lrigw_ctx *c, const char *stage, long long *launches) {
  if (!c || !stage) return -1.0;
  auto it = c->stages.find(stage);
  if (it == c->stages.end()) {
    if (launches) *launches = 0;
    return -1.0;
  }
  StageTimer &t = it->second;
  if (!t.pending.empty()) {
    hipStreamSynchronize(c->stream);
    for (auto &pr : t.pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) t.ms += ms;
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
    t.pending.clear();
  }
  if (launches) *launches = t.launches;
  return t.ms;
}

void lrigw_reset_timing(lrigw_ctx *c) {
  if (!c) return;
  hipStreamSynchronize(c->stream);
  for (auto &kv : c->stages)
    for (auto &pr : kv.second.pending) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  c->stages.clear();
}

}  // extern "C"
