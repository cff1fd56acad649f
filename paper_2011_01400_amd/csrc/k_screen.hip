// Screening (Eqs. symm_dielec_func, screened_W_matr), correlation part, FP64:
//   V = L L^H (Cholesky, once per q)
//   D = -L^H chi L          (eps~ - I, Hermitian positive semidefinite)
//   E = I + D = L_E L_E^H   (batched over frequencies)
//   W^c = L (E^{-1} - I) L^H = -L (E^{-1} D) L^H,   E^{-1} D by two triangular solves
// Using L in place of V^{1/2} leaves W unchanged (L = V^{1/2} Q with Q unitary),
// and E^{-1} D avoids the cancellation of E^{-1} - I where screening is weak.
//
// Truncated Coulomb matrix (Sec. III B): V^cut replaces V in the numerator
// only, W^c = S_c (eps~^{-1} - I) S_c with S = V^{1/2}, S_c = V^cut^{1/2} the
// Hermitian roots and eps~ from the full V.  Since eps~^{-1} - I =
// S L^{-H} (E^{-1} - I) L^{-1} S, this is T (E^{-1} - I) T^H with
// T = S_c S L^{-H}; the screening keeps its Cholesky steps and takes T in
// place of L in the last two products (T = L when V^cut = V).  The two roots
// come from the coupled Newton-Schulz iteration on the FP64 MFMA GEMM,
// Y <- Y M, Z <- M Z, M = (3I - Z Y)/2 from Y = A/|A|_F, Z = I
// (Y -> (A/|A|_F)^{1/2}; a fixed NS_ITERS steps reach FP64 rounding for
// |A|_F / lambda_min up to 1e10).
#include <algorithm>
#include <climits>

#include "lrigw_internal.h"
#include "tiles.h"

template <typename CIN>
__global__ void k_widen(const CIN *__restrict__ in, double2 *__restrict__ out, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) out[i] = to_z(in[i]);
}

// E = I + D
__global__ void k_add_identity(const double2 *__restrict__ D, double2 *__restrict__ E, int n, long long stride) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  long long o = (long long)blockIdx.y * stride + idx;
  double2 v = D[o];
  if (idx / n == idx % n) v.x += 1.0;
  E[o] = v;
}

// out = the Hermitian matrix whose lower triangle (diagonal included) is that
// of W, in the compute type (the diagonal's imaginary part is dropped)
template <typename T>
__global__ void k_hermitize(const double2 *__restrict__ W, typename c2t<T>::type *__restrict__ out, int n, long long stride) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  int r = (int)(idx / n), cc = (int)(idx % n);
  const double2 *Wb = W + (long long)blockIdx.y * stride;
  double2 z;
  if (cc < r) z = Wb[(long long)r * n + cc];
  else if (cc > r) z = cconj(Wb[(long long)cc * n + r]);
  else z = mkc(Wb[(long long)r * n + r].x, 0.0);
  out[(long long)blockIdx.y * stride + idx] = to_c<T>(z);
}

// A[cc][r] = conj(A[r][cc]) for cc > r (upper triangle from the lower one)
__global__ void k_mirror_lower(double2 *A, int n, long long stride) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  int r = (int)(idx / n), cc = (int)(idx % n);
  if (cc <= r) return;
  double2 *Ab = A + (long long)blockIdx.y * stride;
  Ab[(long long)r * n + cc] = cconj(Ab[(long long)cc * n + r]);
}

// sticky status of a captured pass: d_info[16] = smallest q whose V or eps~ was
// not positive definite (INT_MAX: none)
__global__ void k_fold_status(int *info, int q) {
  if (threadIdx.x != 0) return;
  if (info[1] != INT_MAX || info[2] != INT_MAX) info[16] = min(info[16], q);
}

// nrm[b] = Frobenius norm of matrix b (one workgroup per matrix, FP64 sum)
__global__ __launch_bounds__(256) void k_fro_norm(const double2 *__restrict__ A, long long nn, double *__restrict__ nrm) {
  __shared__ double red[256];
  const double2 *a = A + (long long)blockIdx.x * nn;
  double s = 0.0;
  for (long long i = threadIdx.x; i < nn; i += 256) s += a[i].x * a[i].x + a[i].y * a[i].y;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) nrm[blockIdx.x] = sqrt(red[0]);
}

// Y = A / nrm, Z = I (batch element blockIdx.y)
__global__ void k_ns_init(const double2 *__restrict__ A, const double *__restrict__ nrm, double2 *__restrict__ Y,
                          double2 *__restrict__ Z, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nn = (long long)n * n;
  if (idx >= nn) return;
  const long long o = (long long)blockIdx.y * nn + idx;
  const double f = 1.0 / nrm[blockIdx.y];
  const double2 a = A[o];
  Y[o] = mkc(a.x * f, a.y * f);
  Z[o] = mkc(idx / n == idx % n ? 1.0 : 0.0, 0.0);
}

// G <- 1.5 I - 0.5 G
__global__ void k_ns_step(double2 *__restrict__ G, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nn = (long long)n * n;
  if (idx >= nn) return;
  const long long o = (long long)blockIdx.y * nn + idx;
  double2 g = G[o];
  g.x = (idx / n == idx % n ? 1.5 : 0.0) - 0.5 * g.x;
  g.y = -0.5 * g.y;
  G[o] = g;
}

// out = sqrt(nrm) Y
__global__ void k_ns_finish(const double2 *__restrict__ Y, const double *__restrict__ nrm, double2 *__restrict__ out, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nn = (long long)n * n;
  if (idx >= nn) return;
  const long long o = (long long)blockIdx.y * nn + idx;
  const double f = sqrt(nrm[blockIdx.y]);
  out[o] = mkc(Y[o].x * f, Y[o].y * f);
}

#define NS_ITERS 36

static ZGemm mk(int m, int n, int k, int opa, const double2 *A, long long lda, long long sa, int opb, const double2 *B,
                long long ldb, long long sb, double2 *Cm, long long ldc, long long sc, double2 alpha, int batch) {
  ZGemm g;
  g.m = m; g.n = n; g.k = k;
  g.opa = opa; g.A = A; g.lda = lda; g.sa = sa;
  g.opb = opb; g.B = B; g.ldb = ldb; g.sb = sb;
  g.C = Cm; g.ldc = ldc; g.sc = sc;
  g.alpha = alpha; g.beta = mkc(0.0, 0.0);
  g.batch = batch; g.lower_only = 0;
  return g;
}

// Hermitian square roots of the `batch` HPD matrices A[b] (n x n, contiguous)
// into out[b], by the coupled Newton-Schulz iteration; w: 4 batch n^2 + 64
// doubles of workspace (Y, Z, G and a second Y/Z pair; norms at the end).
static int zsqrt_hpd_batched(hipStream_t s, const double2 *A, int n, int batch, double2 *out, double2 *w) {
  const long long nn = (long long)n * n;
  double2 *Y = w, *Z = w + batch * nn, *G = w + 2 * batch * nn, *Y2 = w + 3 * batch * nn, *Z2 = out;
  double *nrm = (double *)(w + 4 * batch * nn);
  const double2 one = mkc(1.0, 0.0);
  hipLaunchKernelGGL(k_fro_norm, dim3(batch), dim3(256), 0, s, A, nn, nrm);
  dim3 eg((unsigned)((nn + 255) / 256), batch);
  hipLaunchKernelGGL(k_ns_init, eg, dim3(256), 0, s, A, nrm, Y, Z, n);
  for (int it = 0; it < NS_ITERS; ++it) {
    LRIGW_TRY(zgemm(s, mk(n, n, n, OP_N, Z, n, nn, OP_N, Y, n, nn, G, n, nn, one, batch)));
    hipLaunchKernelGGL(k_ns_step, eg, dim3(256), 0, s, G, n);
    LRIGW_TRY(zgemm(s, mk(n, n, n, OP_N, Y, n, nn, OP_N, G, n, nn, Y2, n, nn, one, batch)));
    LRIGW_TRY(zgemm(s, mk(n, n, n, OP_N, G, n, nn, OP_N, Z, n, nn, Z2, n, nn, one, batch)));
    std::swap(Y, Y2);
    std::swap(Z, Z2);
  }
  // after an even number of steps Z is back in the workspace and `out` is free
  static_assert(NS_ITERS % 2 == 0, "the last Z must not sit in out");
  hipLaunchKernelGGL(k_ns_finish, eg, dim3(256), 0, s, Y, nrm, out, n);
  return lrigw_launch_check("zsqrt_hpd");
}

// c->d_cut[0] = L^{-1} S S_c (= T^H), with L the Cholesky factor of V in c->d_LV
// and its diagonal-block inverses in c->d_dinv (batch element 0)
static int cut_factor(lrigw_ctx *c, const void *V, const void *Vcut) {
  const int n = c->d.n_aux;
  const long long nn = (long long)n * n;
  hipStream_t s = c->stream;
  // T^H, [V, V^cut], their roots, the root iteration's workspace (8 n^2 + norms)
  if (!c->d_cut) LRIGW_HIP_TRY(hipMalloc(&c->d_cut, (size_t)(13 * nn + 64) * sizeof(double2)));
  double2 *A = c->d_cut + nn, *R = A + 2 * nn, *w = R + 2 * nn;   // [V, V^cut], their roots, workspace
  LRIGW_HIP_TRY(hipMemcpyAsync(A, V, nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
  LRIGW_HIP_TRY(hipMemcpyAsync(A + nn, Vcut, nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
  LRIGW_TRY(zsqrt_hpd_batched(s, A, n, 2, R, w));
  // S S_c, then L^{-1} (S S_c)
  LRIGW_TRY(zgemm(s, mk(n, n, n, OP_N, R, n, 0, OP_N, R + nn, n, 0, c->d_cut, n, 0, mkc(1.0, 0.0), 1)));
  return ztrsm_left_lower(s, c->d_LV, n, nn, c->d_dinv, c->d_cut, n, nn, n, n, 1);
}

// d_info[16] = min(d_info[16], q0 + b) for the first batch element b whose
// factorisation failed (d_info[1]); d_info[1] is reset
__global__ void k_fold_first(int *info, int q0) {
  if (threadIdx.x != 0) return;
  if (info[1] != INT_MAX) {
    info[16] = min(info[16], q0 + info[1]);
    info[1] = INT_MAX;
  }
}

int coulomb_factors(lrigw_ctx *c, const void *V, const void *Vcut, int q0, int q1) {
  c->cf_on = false;
  const int n = c->d.n_aux;
  const long long nn = (long long)n * n, ds = zdinv_stride(n);
  const int nq = q1 - q0;
  if (!V || nq < 1) return LRIGW_ERR_ARG;
  const bool cut = Vcut != nullptr && Vcut != V;
  const int qa = std::max(q0, 1), ncut = cut ? std::max(0, q1 - qa) : 0;
  // root chunks: [V, V^cut] pairs of qc q, roots, workspace (12 qc N^2 + 64), at most 1 GiB
  const int qc = ncut > 0 ? (int)std::max<long long>(1, std::min<long long>(ncut, ((1ll << 30) / 16 - 64) / (12 * nn))) : 0;
  const size_t need = ((size_t)nq * nn * (cut ? 2 : 1) + (size_t)nq * ds + (qc > 0 ? (size_t)12 * qc * nn + 64 : 0)) *
                      sizeof(double2);
  if (need > c->cf_bytes) {
    if (c->d_cf) LRIGW_HIP_TRY(hipFree(c->d_cf));
    c->d_cf = nullptr;
    c->cf_bytes = 0;
    LRIGW_HIP_TRY(hipMalloc(&c->d_cf, need));
    c->cf_bytes = need;
  }
  hipStream_t s = c->stream;
  double2 *L = c->d_cf, *TH = L + (long long)nq * nn, *Dinv = TH + (cut ? (long long)nq * nn : 0);
  double2 *work = Dinv + (long long)nq * ds;
  LRIGW_HIP_TRY(hipMemcpyAsync(L, (const double2 *)V + (long long)q0 * nn, (size_t)nq * nn * sizeof(double2),
                               hipMemcpyDeviceToDevice, s));
  LRIGW_TRY(zpotrf_batched(s, L, n, n, nn, nq, Dinv, c->d_info + 1));
  hipLaunchKernelGGL(k_fold_first, dim3(1), dim3(1), 0, s, c->d_info, q0);
  LRIGW_TRY(lrigw_launch_check("coulomb_factors"));
  // T^H(q) = L^{-1} S S_c for q > 0, qc q at a time
  for (int qb = qa; cut && qb < q1; qb += qc) {
    const int m = std::min(qc, q1 - qb);
    double2 *A = work, *R = A + 2ll * m * nn, *w = R + 2ll * m * nn;
    LRIGW_HIP_TRY(hipMemcpyAsync(A, (const double2 *)V + (long long)qb * nn, (size_t)m * nn * sizeof(double2),
                                 hipMemcpyDeviceToDevice, s));
    LRIGW_HIP_TRY(hipMemcpyAsync(A + (long long)m * nn, (const double2 *)Vcut + (long long)qb * nn,
                                 (size_t)m * nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
    LRIGW_TRY(zsqrt_hpd_batched(s, A, n, 2 * m, R, w));
    double2 *T = TH + (long long)(qb - q0) * nn;
    LRIGW_TRY(zgemm(s, mk(n, n, n, OP_N, R, n, nn, OP_N, R + (long long)m * nn, n, nn, T, n, nn, mkc(1.0, 0.0), m)));
    LRIGW_TRY(ztrsm_left_lower(s, L + (long long)(qb - q0) * nn, n, nn, Dinv + (long long)(qb - q0) * ds, T, n, nn, n, n,
                               m));
  }
  c->cf_V = V;
  c->cf_Vcut = cut ? Vcut : nullptr;
  c->cf_cut = cut;
  c->cf_q0 = q0;
  c->cf_q1 = q1;
  c->cf_on = true;
  return LRIGW_OK;
}

// The factors of the screening of q: L (V = L L^H) and, with V^cut, T^H,
// from the pass's batched factorisation when it covers these matrices, else
// computed here (d_LV, d_cut; V's status in d_info[1]).
static int screen_factors(lrigw_ctx *c, int iq, const void *V, const void *Vcut, const double2 **L, const double2 **TH) {
  const int n = c->d.n_aux;
  const long long nn = (long long)n * n;
  const bool cut = Vcut != nullptr && Vcut != V;
  if (c->cf_on && iq >= c->cf_q0 && iq < c->cf_q1 && V == (const void *)((const double2 *)c->cf_V + (long long)iq * nn) &&
      (!cut || (c->cf_cut && iq > 0 && Vcut == (const void *)((const double2 *)c->cf_Vcut + (long long)iq * nn)))) {
    const int nq = c->cf_q1 - c->cf_q0;
    *L = c->d_cf + (long long)(iq - c->cf_q0) * nn;
    *TH = cut ? c->d_cf + (long long)(nq + iq - c->cf_q0) * nn : nullptr;
    return LRIGW_OK;
  }
  hipStream_t s = c->stream;
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_LV, V, nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
  LRIGW_TRY(zpotrf_batched(s, c->d_LV, n, n, nn, 1, c->d_dinv, c->d_info + 1));
  // T^H = L^{-1} V^{1/2} V^cut^{1/2} (before the dielectric Cholesky reuses d_dinv)
  if (cut) LRIGW_TRY(cut_factor(c, V, Vcut));
  *L = c->d_LV;
  *TH = cut ? c->d_cut : nullptr;
  return LRIGW_OK;
}

int run_screen(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info) {
  return run_screen_n(c, iq, chi, V, Vcut, Wc_out, info, c->d.n_freq);
}

// the first nw <= N_w planes of chi (the workspaces hold N_w)
int run_screen_n(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info, int nw) {
  const Dims &d = c->d;
  const int n = d.n_aux;
  const long long nn = (long long)n * n;
  hipStream_t s = c->stream;
  const bool cut = Vcut != nullptr && Vcut != V;
  const double2 *LV = nullptr, *TH = nullptr;
  LRIGW_TRY(screen_factors(c, iq, V, Vcut, &LV, &TH));
  // chi in FP64
  const double2 *chiz;
  if (c->precision == LRIGW_FP64) {
    chiz = (const double2 *)chi;
  } else {
    long long tot = nw * nn;
    hipLaunchKernelGGL(k_widen<float2>, dim3((unsigned)std::min<long long>((tot + 255) / 256, 16384)), dim3(256), 0, s,
                       (const float2 *)chi, c->d_s3, tot);
    chiz = c->d_s3;
  }
  const double2 one = mkc(1.0, 0.0), mone = mkc(-1.0, 0.0);
  // T1 = chi L ; D = -L^H T1 (Hermitian: lower tiles, then mirrored); L is
  // lower triangular with its upper part zero, so each tile runs only the K
  // range L or L^H leaves nonzero
  ZGemm gt = mk(n, n, n, OP_N, chiz, n, nn, OP_N, LV, n, 0, c->d_s0, n, nn, one, nw);
  gt.tri_b = TRI_LOWER;
  LRIGW_TRY(zgemm(s, gt));
  ZGemm gd = mk(n, n, n, OP_C, LV, n, 0, OP_N, c->d_s0, n, nn, c->d_s1, n, nn, mone, nw);
  gd.lower_only = 1;
  gd.tri_a = TRI_UPPER;
  LRIGW_TRY(zgemm(s, gd));
  dim3 eg((unsigned)((nn + 255) / 256), nw);
  hipLaunchKernelGGL(k_mirror_lower, eg, dim3(256), 0, s, c->d_s1, n, nn);
  // E = I + D, Cholesky
  hipLaunchKernelGGL(k_add_identity, eg, dim3(256), 0, s, c->d_s1, c->d_s2, n, nn);
  LRIGW_TRY(zpotrf_batched(s, c->d_s2, n, n, nn, nw, c->d_dinv, c->d_info + 2));
  // D <- E^{-1} D
  LRIGW_TRY(ztrsm_left_lower(s, c->d_s2, n, nn, c->d_dinv, c->d_s1, n, nn, n, n, nw));
  LRIGW_TRY(ztrsm_left_upper_conj(s, c->d_s2, n, nn, c->d_dinv, c->d_s1, n, nn, n, n, nw));
  // W = -L (E^{-1} D) L^H (Hermitian: lower tiles; k_hermitize mirrors them);
  // with V^cut, T = (T^H)^H in place of L
  if (cut) {
    LRIGW_TRY(zgemm(s, mk(n, n, n, OP_N, c->d_s1, n, nn, OP_N, TH, n, 0, c->d_s0, n, nn, one, nw)));
  } else {
    ZGemm g1 = mk(n, n, n, OP_N, c->d_s1, n, nn, OP_C, LV, n, 0, c->d_s0, n, nn, one, nw);
    g1.tri_b = TRI_UPPER;
    LRIGW_TRY(zgemm(s, g1));
  }
  ZGemm gw = cut ? mk(n, n, n, OP_C, TH, n, 0, OP_N, c->d_s0, n, nn, c->d_s1, n, nn, mone, nw)
                 : mk(n, n, n, OP_N, LV, n, 0, OP_N, c->d_s0, n, nn, c->d_s1, n, nn, mone, nw);
  gw.lower_only = 1;
  if (!cut) gw.tri_a = TRI_LOWER;
  LRIGW_TRY(zgemm(s, gw));
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_hermitize<double>, eg, dim3(256), 0, s, c->d_s1, (double2 *)Wc_out, n, nn);
  else
    hipLaunchKernelGGL(k_hermitize<float>, eg, dim3(256), 0, s, c->d_s1, (float2 *)Wc_out, n, nn);
  LRIGW_TRY(lrigw_launch_check("screen"));
  if (c->capturing) {
    hipLaunchKernelGGL(k_fold_status, dim3(1), dim3(1), 0, s, c->d_info, iq);
    if (info) *info = -1;
    return lrigw_launch_check("screen_status");
  }
  // status: V and eps~ must have been positive definite
  int h[2];
  LRIGW_HIP_TRY(hipMemcpyAsync(h, c->d_info + 1, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  LRIGW_HIP_TRY(hipStreamSynchronize(s));
  if (info) *info = -1;
  if (h[0] != INT_MAX) {
    if (info) *info = -2;
    return LRIGW_ERR_NOT_HPD;
  }
  if (h[1] != INT_MAX) {
    if (info) *info = h[1];
    return LRIGW_ERR_NOT_HPD;
  }
  return LRIGW_OK;
}

// d_info[16] = min(d_info[16], q0 + b / nw) for the first failing batch
// element b of a grouped eps~ factorisation (d_info[2]); d_info[2] is reset
__global__ void k_fold_group(int *info, int q0, int nw) {
  if (threadIdx.x != 0) return;
  if (info[2] != INT_MAX) {
    info[16] = min(info[16], q0 + info[2] / nw);
    info[2] = INT_MAX;
  }
}

long long group_ws_elems(const lrigw_ctx *c, int nq) {
  const long long nn = (long long)c->d.n_aux * c->d.n_aux, nb = (long long)nq * c->d.n_freq;
  return 4 * nb * nn + nb * zdinv_stride(c->d.n_aux);
}

int run_screen_group(lrigw_ctx *c, int q0, int nq, const void *chi, const void *V, const void *Vcut, void *Wc_out,
                     double2 *ws) {
  const Dims &d = c->d;
  const int n = d.n_aux, nw = d.n_freq;
  const long long nn = (long long)n * n, nb = (long long)nq * nw;
  hipStream_t s = c->stream;
  const bool cut = Vcut != nullptr && Vcut != V;
  // the pass's factors: L(q) (and T^H(q)) at a stride of N^2 from q0
  if (!c->cf_on || q0 < c->cf_q0 || q0 + nq > c->cf_q1 || V != (const void *)((const double2 *)c->cf_V + (long long)q0 * nn) ||
      (cut && (!c->cf_cut || q0 < 1 || Vcut != (const void *)((const double2 *)c->cf_Vcut + (long long)q0 * nn))))
    return LRIGW_ERR_ARG;
  const int nqc = c->cf_q1 - c->cf_q0;
  const double2 *LV = c->d_cf + (long long)(q0 - c->cf_q0) * nn;
  const double2 *TH = cut ? c->d_cf + (long long)(nqc + q0 - c->cf_q0) * nn : nullptr;
  double2 *s0 = ws, *s1 = s0 + nb * nn, *s2 = s1 + nb * nn, *s3 = s2 + nb * nn, *dinv = s3 + nb * nn;
  const double2 *chiz;
  if (c->precision == LRIGW_FP64) {
    chiz = (const double2 *)chi;
  } else {
    const long long tot = nb * nn;
    hipLaunchKernelGGL(k_widen<float2>, dim3((unsigned)std::min<long long>((tot + 255) / 256, 16384)), dim3(256), 0, s,
                       (const float2 *)chi, s3, tot);
    chiz = s3;
  }
  const double2 one = mkc(1.0, 0.0), mone = mkc(-1.0, 0.0);
  // the same steps as run_screen_n over nq N_w planes; the factor of plane b
  // is that of q0 + b / N_w (element b of an operand is read at
  // (b % N_w) s + (b / N_w) s2: the factor has s = 0, s2 = N^2, the other
  // operand its plane stride s and s2 = N_w s)
  auto per_q = [&](ZGemm g, bool a_is_factor) {
    g.bdiv = nw;
    if (a_is_factor) {
      g.sa2 = nn;
      g.sb2 = (long long)nw * g.sb;
    } else {
      g.sb2 = nn;
      g.sa2 = (long long)nw * g.sa;
    }
    return g;
  };
  ZGemm gt = per_q(mk(n, n, n, OP_N, chiz, n, nn, OP_N, LV, n, 0, s0, n, nn, one, (int)nb), false);
  gt.tri_b = TRI_LOWER;
  LRIGW_TRY(zgemm(s, gt));
  ZGemm gd = per_q(mk(n, n, n, OP_C, LV, n, 0, OP_N, s0, n, nn, s1, n, nn, mone, (int)nb), true);
  gd.lower_only = 1;
  gd.tri_a = TRI_UPPER;
  LRIGW_TRY(zgemm(s, gd));
  dim3 eg((unsigned)((nn + 255) / 256), (unsigned)nb);
  hipLaunchKernelGGL(k_mirror_lower, eg, dim3(256), 0, s, s1, n, nn);
  hipLaunchKernelGGL(k_add_identity, eg, dim3(256), 0, s, s1, s2, n, nn);
  LRIGW_TRY(zpotrf_batched(s, s2, n, n, nn, (int)nb, dinv, c->d_info + 2));
  hipLaunchKernelGGL(k_fold_group, dim3(1), dim3(1), 0, s, c->d_info, q0, nw);
  LRIGW_TRY(ztrsm_left_lower(s, s2, n, nn, dinv, s1, n, nn, n, n, (int)nb));
  LRIGW_TRY(ztrsm_left_upper_conj(s, s2, n, nn, dinv, s1, n, nn, n, n, (int)nb));
  if (cut) {
    LRIGW_TRY(zgemm(s, per_q(mk(n, n, n, OP_N, s1, n, nn, OP_N, TH, n, 0, s0, n, nn, one, (int)nb), false)));
  } else {
    ZGemm g1 = per_q(mk(n, n, n, OP_N, s1, n, nn, OP_C, LV, n, 0, s0, n, nn, one, (int)nb), false);
    g1.tri_b = TRI_UPPER;
    LRIGW_TRY(zgemm(s, g1));
  }
  ZGemm gw = cut ? per_q(mk(n, n, n, OP_C, TH, n, 0, OP_N, s0, n, nn, s1, n, nn, mone, (int)nb), true)
                 : per_q(mk(n, n, n, OP_N, LV, n, 0, OP_N, s0, n, nn, s1, n, nn, mone, (int)nb), true);
  gw.lower_only = 1;
  if (!cut) gw.tri_a = TRI_LOWER;
  LRIGW_TRY(zgemm(s, gw));
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_hermitize<double>, eg, dim3(256), 0, s, s1, (double2 *)Wc_out, n, nn);
  else
    hipLaunchKernelGGL(k_hermitize<float>, eg, dim3(256), 0, s, s1, (float2 *)Wc_out, n, nn);
  return lrigw_launch_check("screen_group");
}

// ---------------------------------------------------------------- complex frequencies
// out[p] = chi[2p] + i chi[2p+1] in FP64 (the Re- and Im-weight planes of the
// response at w_r + i eta, each a Hermitian matrix)
template <typename C>
__global__ void k_combine_planes(const C *__restrict__ chi, double2 *__restrict__ out, long long nn) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn) return;
  const int p = blockIdx.y;
  const double2 a = to_z(chi[(2LL * p) * nn + idx]), b = to_z(chi[(2LL * p + 1) * nn + idx]);
  out[(long long)p * nn + idx] = mkc(a.x - b.y, a.y + b.x);
}

// out = (W + W^H)/2 in the compute type
template <typename T>
__global__ void k_herm_part(const double2 *__restrict__ W, typename c2t<T>::type *__restrict__ out, int n, long long stride) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  const int r = (int)(idx / n), cc = (int)(idx % n);
  const double2 *Wb = W + (long long)blockIdx.y * stride;
  const double2 a = Wb[(long long)r * n + cc], b = Wb[(long long)cc * n + r];
  double2 z = mkc(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  if (r == cc) z.y = 0.0;
  out[(long long)blockIdx.y * stride + idx] = to_c<T>(z);
}

// Screening at complex frequencies z_p = w_p + i eta, p < np: chi holds 2 np
// planes (the Re- and Im-weight responses of each z_p, compute type).  eps~ is
// not Hermitian there: with D = -L^H chi L and E = I + D (general), E^{-1} D
// comes from the Hermitian positive definite normal equations
// (E^H E) X = E^H D, on the batched Cholesky and triangular solves (in FP64 the
// squared condition number of E, ~1/eta^2 near a resonance, leaves ~1e-10);
// W^c = -L X L^H (or T with V^cut), and Wh_out receives its Hermitian part
// (W + W^H)/2, whose quadratic forms are Re X_nm (the part Re Sigma^c takes).
int run_screen_cplx(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wh_out, int *info,
                    int np) {
  const Dims &d = c->d;
  const int n = d.n_aux;
  const long long nn = (long long)n * n;
  hipStream_t s = c->stream;
  if (np < 1 || np > d.n_freq) return LRIGW_ERR_ARG;
  const bool cut = Vcut != nullptr && Vcut != V;
  const double2 *LV = nullptr, *TH = nullptr;
  LRIGW_TRY(screen_factors(c, iq, V, Vcut, &LV, &TH));
  dim3 eg((unsigned)((nn + 255) / 256), np);
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_combine_planes<double2>, eg, dim3(256), 0, s, (const double2 *)chi, c->d_s3, nn);
  else
    hipLaunchKernelGGL(k_combine_planes<float2>, eg, dim3(256), 0, s, (const float2 *)chi, c->d_s3, nn);
  const double2 one = mkc(1.0, 0.0), mone = mkc(-1.0, 0.0);
  // T1 = chi L; D = -L^H T1 (full: not Hermitian)
  {
    ZGemm gt = mk(n, n, n, OP_N, c->d_s3, n, nn, OP_N, LV, n, 0, c->d_s0, n, nn, one, np);
    gt.tri_b = TRI_LOWER;
    LRIGW_TRY(zgemm(s, gt));
    ZGemm gd = mk(n, n, n, OP_C, LV, n, 0, OP_N, c->d_s0, n, nn, c->d_s1, n, nn, mone, np);
    gd.tri_a = TRI_UPPER;
    LRIGW_TRY(zgemm(s, gd));
  }
  // E = I + D; G = E^H E, R = E^H D
  hipLaunchKernelGGL(k_add_identity, eg, dim3(256), 0, s, c->d_s1, c->d_s2, n, nn);
  LRIGW_TRY(zgemm(s, mk(n, n, n, OP_C, c->d_s2, n, nn, OP_N, c->d_s2, n, nn, c->d_s0, n, nn, one, np)));
  LRIGW_TRY(zgemm(s, mk(n, n, n, OP_C, c->d_s2, n, nn, OP_N, c->d_s1, n, nn, c->d_s3, n, nn, one, np)));
  // X = G^{-1} R = E^{-1} D
  LRIGW_TRY(zpotrf_batched(s, c->d_s0, n, n, nn, np, c->d_dinv, c->d_info + 2));
  LRIGW_TRY(ztrsm_left_lower(s, c->d_s0, n, nn, c->d_dinv, c->d_s3, n, nn, n, n, np));
  LRIGW_TRY(ztrsm_left_upper_conj(s, c->d_s0, n, nn, c->d_dinv, c->d_s3, n, nn, n, n, np));
  // W = -L X L^H (T in place of L with V^cut), full
  if (cut) {
    LRIGW_TRY(zgemm(s, mk(n, n, n, OP_N, c->d_s3, n, nn, OP_N, TH, n, 0, c->d_s1, n, nn, one, np)));
    LRIGW_TRY(zgemm(s, mk(n, n, n, OP_C, TH, n, 0, OP_N, c->d_s1, n, nn, c->d_s2, n, nn, mone, np)));
  } else {
    ZGemm g1 = mk(n, n, n, OP_N, c->d_s3, n, nn, OP_C, LV, n, 0, c->d_s1, n, nn, one, np);
    g1.tri_b = TRI_UPPER;
    LRIGW_TRY(zgemm(s, g1));
    ZGemm g2 = mk(n, n, n, OP_N, LV, n, 0, OP_N, c->d_s1, n, nn, c->d_s2, n, nn, mone, np);
    g2.tri_a = TRI_LOWER;
    LRIGW_TRY(zgemm(s, g2));
  }
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_herm_part<double>, eg, dim3(256), 0, s, c->d_s2, (double2 *)Wh_out, n, nn);
  else
    hipLaunchKernelGGL(k_herm_part<float>, eg, dim3(256), 0, s, c->d_s2, (float2 *)Wh_out, n, nn);
  LRIGW_TRY(lrigw_launch_check("screen_cplx"));
  if (c->capturing) {
    hipLaunchKernelGGL(k_fold_status, dim3(1), dim3(1), 0, s, c->d_info, iq);
    if (info) *info = -1;
    return lrigw_launch_check("screen_status");
  }
  int h[2];
  LRIGW_HIP_TRY(hipMemcpyAsync(h, c->d_info + 1, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  LRIGW_HIP_TRY(hipStreamSynchronize(s));
  if (info) *info = -1;
  if (h[0] != INT_MAX) {
    if (info) *info = -2;
    return LRIGW_ERR_NOT_HPD;
  }
  if (h[1] != INT_MAX) {
    if (info) *info = h[1];
    return LRIGW_ERR_NOT_HPD;
  }
  return LRIGW_OK;
}

// out = tmp * w (first direction) or out + tmp * w
template <typename C>
__global__ void k_waccum(C *__restrict__ out, const C *__restrict__ tmp, long long n, double w, int first) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    C t = tmp[i], o = first ? C{0, 0} : out[i];
    o.x += w * t.x;
    o.y += w * t.y;
    out[i] = o;
  }
}

// W^c(q -> 0) averaged over the context's directions: per direction the q = 0
// response with that direction's head and wings (M already built for q = 0),
// its screening into tmp, and out = sum_d w_d tmp_d.  Runs on c->stream; the
// screening status follows c->capturing as in run_screen.
int run_gamma_average(lrigw_ctx *c, const double *eig, const void *V0, bool real_axis, void *chi, void *tmp, void *out) {
  const Dims &d = c->d;
  const int nw = real_axis ? c->n_real : d.n_freq;
  const long long n = (long long)nw * d.n_aux * d.n_aux;
  const size_t per = (size_t)lrigw_K(c);
  const void *saved = c->gamma_p;
  const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 16384);
  int rc = LRIGW_OK;
  for (int g = 0; g < c->n_gdir && rc == LRIGW_OK; ++g) {
    c->gamma_p = (const double2 *)c->gdir_p + g * per;
    rc = real_axis ? run_chi0_real(c, 0, c->d_M, eig, 1, chi) : run_chi0(c, 0, c->d_M, eig, 1, chi);
    if (rc == LRIGW_OK) rc = run_screen_n(c, 0, chi, V0, nullptr, tmp, nullptr, nw);
    if (rc != LRIGW_OK) break;
    if (c->precision == LRIGW_FP64)
      hipLaunchKernelGGL(k_waccum<double2>, dim3(nb), dim3(256), 0, c->stream, (double2 *)out, (const double2 *)tmp, n,
                         c->gdir_w[g], g == 0 ? 1 : 0);
    else
      hipLaunchKernelGGL(k_waccum<float2>, dim3(nb), dim3(256), 0, c->stream, (float2 *)out, (const float2 *)tmp, n,
                         c->gdir_w[g], g == 0 ? 1 : 0);
    rc = lrigw_launch_check("gamma_average");
  }
  c->gamma_p = saved;
  return rc;
}

