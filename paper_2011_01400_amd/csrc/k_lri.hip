// LRI Bloch transform (Sec. II C, Eqs. expan_coeff_FT1/2) and half-transform
// H[k][a][n][mu] = sum_j C~^{mu(0)}_{a(0), j(k)} c_{j n}(k).
#include <algorithm>

#include "lrigw_internal.h"
#include "tiles.h"

// exp(2 pi i k.R) for the grid points k0..k0+nkc-1; the phase is reduced as an
// exact rational t / (n1 n2 n3) of a full turn before sincospi.
__global__ void k_phases(const int *R, int nR, int n1, int n2, int n3, int k0, int nkc, double2 *ph) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nkc * nR) return;
  int kk = idx / nR, r = idx % nR;
  int k = k0 + kk;
  int i1 = k / (n2 * n3), i2 = (k / n3) % n2, i3 = k % n3;
  long long nt = (long long)n1 * n2 * n3;
  long long t = (long long)i1 * R[3 * r] * n2 * n3 + (long long)i2 * R[3 * r + 1] * n1 * n3 + (long long)i3 * R[3 * r + 2] * n1 * n2;
  t %= nt;
  if (t < 0) t += nt;
  double s, c;
  sincospi(2.0 * (double)t / (double)nt, &s, &c);
  ph[idx] = mkc(c, s);
}

// out[kk][e] = sum_R ph[kk][R] * L[R][e] for KCH grid points at once.
template <int KCH>
__global__ __launch_bounds__(256) void k_bloch(const double *__restrict__ L, long long E, int nR, const double2 *__restrict__ ph,
                                               int nkc, double2 *__restrict__ out, long long ldo) {
  extern __shared__ double2 sph[];
  for (int i = threadIdx.x; i < nkc * nR; i += blockDim.x) sph[i] = ph[i];
  __syncthreads();
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  double ar[KCH], ai[KCH];
#pragma unroll
  for (int j = 0; j < KCH; ++j) ar[j] = ai[j] = 0.0;
  for (int r = 0; r < nR; ++r) {
    double v = L[(long long)r * E + e];
#pragma unroll
    for (int j = 0; j < KCH; ++j)
      if (j < nkc) {
        double2 p = sph[j * nR + r];
        ar[j] += p.x * v;
        ai[j] += p.y * v;
      }
  }
#pragma unroll
  for (int j = 0; j < KCH; ++j)
    if (j < nkc) out[(long long)j * ldo + e] = mkc(ar[j], ai[j]);
}

template <typename T>
__global__ void k_to_compute(const double2 *__restrict__ in, typename c2t<T>::type *__restrict__ out, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) out[i] = to_c<T>(in[i]);
}

int run_lri_ft(lrigw_ctx *c, const double *lri_R, const int *R_list, int nR, const void *evec, void *H_out) {
  const Dims &d = c->d;
  const int KCH = 8;
  if ((size_t)KCH * nR * sizeof(double2) > 64 * 1024) return LRIGW_ERR_ARG;  // phases must fit in LDS
  for (int r = 0; r < 3 * nR; ++r)
    if (R_list[r] < -100000 || R_list[r] > 100000) return LRIGW_ERR_ARG;
  const bool f64 = c->precision == LRIGW_FP64;
  std::vector<long long> eoff(d.n_atoms + 1, 0);  // per-atom element offsets, E_A = naux_A * nb_A * N_b
  for (int A = 0; A < d.n_atoms; ++A)
    eoff[A + 1] = eoff[A] + (long long)(c->aux_off[A + 1] - c->aux_off[A]) * (c->basis_off[A + 1] - c->basis_off[A]) * d.n_b;
  const long long Etot = eoff[d.n_atoms];
  const long long hk = (long long)d.nb_max * d.n_bands * d.n_aux;  // H elements per k

  int *dR = nullptr;
  double2 *ph = nullptr, *Lk = nullptr, *Hz = nullptr;
  int rc = LRIGW_OK;
  auto cleanup = [&]() {
    hipStreamSynchronize(c->stream);
    if (dR) (void)hipFree(dR);
    if (ph) (void)hipFree(ph);
    if (Lk) (void)hipFree(Lk);
    if (Hz) (void)hipFree(Hz);
  };
#define FT_TRY(x)                    \
  do {                               \
    hipError_t e__ = (x);            \
    if (e__ != hipSuccess) {         \
      rc = lrigw_hip_error(e__, #x, __FILE__, __LINE__); \
      cleanup();                     \
      return rc;                     \
    }                                \
  } while (0)
  FT_TRY(hipMalloc(&dR, (size_t)3 * nR * sizeof(int)));
  FT_TRY(hipMemcpyAsync(dR, R_list, (size_t)3 * nR * sizeof(int), hipMemcpyHostToDevice, c->stream));
  FT_TRY(hipMalloc(&ph, (size_t)KCH * nR * sizeof(double2)));
  FT_TRY(hipMalloc(&Lk, (size_t)KCH * Etot * sizeof(double2)));
  if (!f64) FT_TRY(hipMalloc(&Hz, (size_t)KCH * hk * sizeof(double2)));
  // rows a >= nb_A of an atom stay zero
  rc = zero_fill(c->stream, f64 ? H_out : Hz, (size_t)(f64 ? d.n_k : KCH) * hk * sizeof(double2));
  if (rc < 0) { cleanup(); return rc; }

  for (int k0 = 0; k0 < d.n_k; k0 += KCH) {
    int nkc = std::min(KCH, d.n_k - k0);
    hipLaunchKernelGGL(k_phases, dim3((nkc * nR + 255) / 256), dim3(256), 0, c->stream, dR, nR, d.nk[0], d.nk[1], d.nk[2],
                       k0, nkc, ph);
    for (int A = 0; A < d.n_atoms; ++A) {
      long long EA = eoff[A + 1] - eoff[A];
      hipLaunchKernelGGL(k_bloch<KCH>, dim3((unsigned)((EA + 255) / 256)), dim3(256), nkc * nR * sizeof(double2), c->stream,
                         lri_R + eoff[A] * nR, EA, nR, ph, nkc, Lk + eoff[A], Etot);
    }
    if ((rc = lrigw_launch_check("lri bloch")) < 0) { cleanup(); return rc; }
    for (int kk = 0; kk < nkc; ++kk) {
      int k = k0 + kk;
      double2 *Hk = f64 ? (double2 *)H_out + (long long)k * hk : Hz + (long long)kk * hk;
      for (int A = 0; A < d.n_atoms; ++A) {
        int nbA = c->basis_off[A + 1] - c->basis_off[A];
        int naA = c->aux_off[A + 1] - c->aux_off[A];
        // for each a of atom A: Hk[a][n][mu_A] = sum_j c[k][j][n] * Lk[kk][A][mu][a][j]
        ZGemm g;
        g.m = d.n_bands;
        g.n = naA;
        g.k = d.n_b;
        g.opa = OP_T;
        g.A = (const double2 *)evec + (long long)k * d.n_b * d.n_bands;
        g.lda = d.n_bands;
        g.sa = 0;
        g.opb = OP_T;
        g.B = Lk + (long long)kk * Etot + eoff[A];
        g.ldb = (long long)nbA * d.n_b;
        g.sb = d.n_b;
        g.C = Hk + c->aux_off[A];
        g.ldc = d.n_aux;
        g.sc = (long long)d.n_bands * d.n_aux;
        g.alpha = mkc(1.0, 0.0);
        g.beta = mkc(0.0, 0.0);
        g.batch = nbA;
        g.lower_only = 0;
        if ((rc = zgemm(c->stream, g)) < 0) { cleanup(); return rc; }
      }
    }
    if (!f64) {
      long long n = (long long)nkc * hk;
      hipLaunchKernelGGL(k_to_compute<float>, dim3((unsigned)std::min<long long>((n + 255) / 256, 16384)), dim3(256), 0,
                         c->stream, Hz, (float2 *)H_out + (long long)k0 * hk, n);
      if ((rc = lrigw_launch_check("lri convert")) < 0) { cleanup(); return rc; }
    }
  }
#undef FT_TRY
  cleanup();
  return LRIGW_OK;
}
