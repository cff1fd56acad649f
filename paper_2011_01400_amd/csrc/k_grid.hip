// Grids: Gauss-Legendre nodes on the device, k+q / k-q tables, workspaces.
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

// Modified Gauss-Legendre grid (Sec. II A works on the imaginary axis; the grid
// maps Gauss-Legendre nodes t in (-1,1) to omega = x0 (1+t)/(1-t)).  Node i in
// ascending order is found by Newton's method on P_n from the Chebyshev-like
// first guess cos(pi (n-1-i+3/4)/(n+1/2)); P_n and P_n' come from the
// three-term recurrence; weight = 2 / ((1-t^2) P_n'(t)^2).
__global__ void k_gauss_legendre(int n, double x0, double *omega, double *weight) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double t = cos(M_PI * ((double)(n - 1 - i) + 0.75) / ((double)n + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = t;
    for (int l = 2; l <= n; ++l) {
      double p2 = ((2.0 * l - 1.0) * t * p1 - (l - 1.0) * p0) / (double)l;
      p0 = p1;
      p1 = p2;
    }
    // p1 = P_n(t), p0 = P_{n-1}(t)
    dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
    double dt = p1 / dp;
    t -= dt;
    if (fabs(dt) < 1e-16) {
      // one more evaluation of the derivative at the converged root
      p0 = 1.0;
      p1 = t;
      for (int l = 2; l <= n; ++l) {
        double p2 = ((2.0 * l - 1.0) * t * p1 - (l - 1.0) * p0) / (double)l;
        p0 = p1;
        p1 = p2;
      }
      dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
      break;
    }
  }
  double g = 2.0 / ((1.0 - t * t) * dp * dp);
  omega[i] = x0 * (1.0 + t) / (1.0 - t);
  weight[i] = g * 2.0 * x0 / ((1.0 - t) * (1.0 - t));
}

__global__ void k_fill_zero(uint32_t *p, long long n_words) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (; i < n_words; i += stride) p[i] = 0u;
}

int zero_fill(hipStream_t s, void *p, size_t bytes) {
  if (bytes == 0) return LRIGW_OK;
  long long words = (long long)(bytes / 4);
  int blocks = (int)std::min<long long>((words + 255) / 256, 8192);
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, words);
  return lrigw_launch_check("fill_zero");
}

static int kindex(const int nk[3], int a, int b, int c) {
  a = ((a % nk[0]) + nk[0]) % nk[0];
  b = ((b % nk[1]) + nk[1]) % nk[1];
  c = ((c % nk[2]) + nk[2]) % nk[2];
  return (a * nk[1] + b) * nk[2] + c;
}

int run_grids(lrigw_ctx *c) {
  Dims &d = c->d;
  const int nk = d.n_k;
  // k tables (integer bookkeeping on the host)
  c->h_kpq.resize((size_t)nk * nk);
  c->h_kmq.resize((size_t)nk * nk);
  std::vector<int> ki(nk * 3);
  for (int a = 0; a < d.nk[0]; ++a)
    for (int b = 0; b < d.nk[1]; ++b)
      for (int e = 0; e < d.nk[2]; ++e) {
        int k = (a * d.nk[1] + b) * d.nk[2] + e;
        ki[3 * k] = a;
        ki[3 * k + 1] = b;
        ki[3 * k + 2] = e;
      }
  for (int k = 0; k < nk; ++k)
    for (int q = 0; q < nk; ++q) {
      c->h_kpq[(size_t)k * nk + q] = kindex(d.nk, ki[3 * k] + ki[3 * q], ki[3 * k + 1] + ki[3 * q + 1], ki[3 * k + 2] + ki[3 * q + 2]);
      c->h_kmq[(size_t)k * nk + q] = kindex(d.nk, ki[3 * k] - ki[3 * q], ki[3 * k + 1] - ki[3 * q + 1], ki[3 * k + 2] - ki[3 * q + 2]);
    }
  std::vector<int> aux_atom(d.n_aux);
  for (int A = 0; A < d.n_atoms; ++A)
    for (int m = c->aux_off[A]; m < c->aux_off[A + 1]; ++m) aux_atom[m] = A;

  size_t kk = (size_t)nk * nk * sizeof(int);
  LRIGW_HIP_TRY(hipMalloc(&c->d_kpq, kk));
  LRIGW_HIP_TRY(hipMalloc(&c->d_kmq, kk));
  LRIGW_HIP_TRY(hipMalloc(&c->d_aux_atom, d.n_aux * sizeof(int)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_basis_off, (d.n_atoms + 1) * sizeof(int)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_aux_off, (d.n_atoms + 1) * sizeof(int)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_omega, d.n_freq * sizeof(double)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_weight, d.n_freq * sizeof(double)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_wall, d.n_freq * sizeof(int)));
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_kpq, c->h_kpq.data(), kk, hipMemcpyHostToDevice, c->stream));
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_kmq, c->h_kmq.data(), kk, hipMemcpyHostToDevice, c->stream));
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_aux_atom, aux_atom.data(), d.n_aux * sizeof(int), hipMemcpyHostToDevice, c->stream));
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_basis_off, c->basis_off.data(), (d.n_atoms + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_aux_off, c->aux_off.data(), (d.n_atoms + 1) * sizeof(int), hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(k_gauss_legendre, dim3((d.n_freq + 63) / 64), dim3(64), 0, c->stream, d.n_freq, d.x0, c->d_omega,
                     c->d_weight);
  LRIGW_TRY(lrigw_launch_check("gauss_legendre"));
  std::vector<int> wall(d.n_freq);
  for (int i = 0; i < d.n_freq; ++i) wall[i] = i;
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_wall, wall.data(), d.n_freq * sizeof(int), hipMemcpyHostToDevice, c->stream));
  c->h_omega.resize(d.n_freq);
  c->h_weight.resize(d.n_freq);
  LRIGW_HIP_TRY(hipMemcpyAsync(c->h_omega.data(), c->d_omega, d.n_freq * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LRIGW_HIP_TRY(hipMemcpyAsync(c->h_weight.data(), c->d_weight, d.n_freq * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));
  // response tables of the imaginary planes (the real-axis half is filled when
  // a real grid is set): w^2, and the FP16 split's scale 2^-e with
  // 2D/(D^2 + w^2) <= 1/w < 2^e
  c->h_om2.assign(2 * (size_t)d.n_freq, 0.0);
  c->h_wsc.assign(2 * (size_t)d.n_freq, 1.f);
  for (int i = 0; i < d.n_freq; ++i) {
    const double o = c->h_omega[i];
    c->h_om2[i] = o * o;
    int e = 0;
    if (o > 0.0) frexp(1.0 / o, &e);
    c->h_wsc[i] = ldexpf(1.f, -e);
  }
  LRIGW_HIP_TRY(hipMalloc(&c->d_om2, c->h_om2.size() * sizeof(double)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_wsc, c->h_wsc.size() * sizeof(float)));
  LRIGW_HIP_TRY(hipMemcpy(c->d_om2, c->h_om2.data(), c->h_om2.size() * sizeof(double), hipMemcpyHostToDevice));
  LRIGW_HIP_TRY(hipMemcpy(c->d_wsc, c->h_wsc.data(), c->h_wsc.size() * sizeof(float), hipMemcpyHostToDevice));

  // workspaces
  const bool f64 = c->precision == LRIGW_FP64;
  const size_t rs = f64 ? sizeof(double) : sizeof(float);
  const size_t cs = lrigw_csize(c);
  const long long K = lrigw_K(c);
  const size_t nn = (size_t)d.n_aux * d.n_aux;
  LRIGW_HIP_TRY(hipMalloc(&c->d_delta, (size_t)K * rs));
  c->chi_nw = chi0_default_nw(c->precision);
  c->sig_var = sigma_default_variant(c->precision);
  LRIGW_TRY(chi0_plan_splits(c, &c->chi_splits));
  c->part_bytes = chi0_part_bytes(c, c->chi_splits);
  LRIGW_HIP_TRY(hipMalloc(&c->d_part, c->part_bytes));
  LRIGW_HIP_TRY(hipMalloc(&c->d_X, (size_t)d.n_freq * d.n_k * d.n_qp * d.n_bands * sizeof(double)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_LV, nn * sizeof(double2)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_s0, d.n_freq * nn * sizeof(double2)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_s1, d.n_freq * nn * sizeof(double2)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_s2, d.n_freq * nn * sizeof(double2)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_s3, d.n_freq * nn * sizeof(double2)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_dinv, (size_t)d.n_freq * zdinv_stride(d.n_aux) * sizeof(double2)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_info, 64 * sizeof(int)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_x1, d.n_aux * sizeof(double2)));
  if (ns_chi(c->precision) > 0) {
    const int NSS = ns_sig(c->precision), NSC = ns_chi(c->precision);
    const long long Ccols = (long long)d.n_k * d.n_qp * d.n_bands;
    const long long Cpad = (Ccols + TILE - 1) / TILE * TILE;
    const long long Npad = (d.n_aux + 31) / 32 * 32;
    const long long Rpad = (d.n_aux + TILE - 1) / TILE * TILE;
    LRIGW_HIP_TRY(hipMalloc(&c->d_xs, (size_t)NSS * 2 * Cpad * Npad * 2));
    LRIGW_HIP_TRY(hipMalloc(&c->d_ws, (size_t)d.n_freq * NSS * 2 * Rpad * Npad * 2));
    const long long Kp = (K + 31) / 32 * 32;
    LRIGW_HIP_TRY(hipMalloc(&c->d_ap, (size_t)NSC * 2 * Rpad * Kp * 2));
    LRIGW_HIP_TRY(hipMalloc(&c->d_bt, (size_t)Rpad * Kp * sizeof(float2)));
    LRIGW_HIP_TRY(hipMalloc(&c->d_sx, (size_t)Cpad * sizeof(float)));
    LRIGW_HIP_TRY(hipMalloc(&c->d_wmax, (size_t)d.n_freq * sizeof(unsigned)));
    LRIGW_HIP_TRY(hipMalloc(&c->d_amax, (size_t)Rpad * sizeof(unsigned)));
    LRIGW_TRY(sigma_res_prepare(c));
  }
  return LRIGW_OK;
}
