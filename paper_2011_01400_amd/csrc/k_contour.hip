// Correlation self-energy at real energies by contour deformation.
//
// Contour deformation is the alternative to analytic continuation that the
// paper names (Sec. II A, after Eq. chi_0_realspace).  Deforming the
// real-axis frequency integral of G W^c onto the imaginary axis leaves that
// integral plus the residues of the Green-function poles passed over.  With
// the pair weights X_nm(k,q,w) = x^T W^c(q,w) conj(x) of Eq. GW_selfe_element
// and z = E - e_m(k-q):
//   Sigma^c_n(k,E) = 1/N_q sum_q sum_m [ -(1/pi) int_0^inf X(iw) z/(z^2+w^2) dw
//                                        + theta_m(E) X(|z|) ],
// theta = +1 for an unoccupied m below E, -1 for an occupied m above E, half
// of that at E = e_m.
//
// W^c on the real axis is formed below the smallest transition energy only.
// There the response weight is 2D/(D^2 - w^2), chi~ is Hermitian and
// eps~ positive definite.  The same kernels build it through the per-plane
// tables (signed w^2 and the FP16 split's scale).  Its planes sit on a uniform
// grid w_r = r h.  X between nodes is the 4-point Lagrange interpolant, with
// the stencil reflected at w = 0 (X is even).  The imaginary-axis integral uses
// the response's own grid with X(0) subtracted and its integral,
// (pi/2) sgn(z) X(0), added in closed form.  X(0) is the real grid's first
// plane.  A residue frequency beyond the grid's top gives NaN.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "lrigw_internal.h"

#define CD_EMAX 4

// sigma_e[e][k][n] += scale * sum_m [ -(1/pi) sum_j g_j (X_j - X_0) z/(z^2 + w_j^2)
//                                     - sgn(z) X_0 / 2 + theta_m X(|z|) ],  z = E[e][k][n] - e_m(k-q)
// One wave per (k, n); lanes run over m (X rows contiguous in m); the lane
// sums are combined by a butterfly in a fixed order.
__global__ __launch_bounds__(64) void k_sigma_cd(const double *__restrict__ X, const double *__restrict__ Xr,
                                                 const double *__restrict__ eig, const int *__restrict__ kmq, int iq, int nk,
                                                 int n_qp, int n_bands, int n_occ, int n_freq,
                                                 const double *__restrict__ omega, const double *__restrict__ weight, int n_r,
                                                 double h, int n_e, const double *__restrict__ E, double scale,
                                                 double *__restrict__ sigma_e) {
  const int k = blockIdx.x / n_qp, n = blockIdx.x % n_qp, lane = threadIdx.x;
  const int k2 = kmq[k * nk + iq];
  const long long cstride = (long long)nk * n_qp * n_bands;
  const long long row = ((long long)k * n_qp + n) * n_bands;
  const double top = (n_r - 1) * h;
  double Ev[CD_EMAX], acc[CD_EMAX];
#pragma unroll
  for (int e = 0; e < CD_EMAX; ++e) {
    Ev[e] = e < n_e ? E[((long long)e * nk + k) * n_qp + n] : 0.0;
    acc[e] = 0.0;
  }
  for (int m = lane; m < n_bands; m += 64) {
    const double em = eig[(long long)k2 * n_bands + m];
    const bool occ = m < n_occ;
    const double *xr = Xr + row + m;
    const double *xi = X + row + m;
    const double X0 = xr[0];
    double z[CD_EMAX], s[CD_EMAX];
#pragma unroll
    for (int e = 0; e < CD_EMAX; ++e) {
      z[e] = Ev[e] - em;
      s[e] = 0.0;
    }
    for (int j = 0; j < n_freq; ++j) {
      const double xd = weight[j] * (xi[(long long)j * cstride] - X0);
      const double w2 = omega[j] * omega[j];
#pragma unroll
      for (int e = 0; e < CD_EMAX; ++e) s[e] += xd * z[e] / (z[e] * z[e] + w2);
    }
#pragma unroll
    for (int e = 0; e < CD_EMAX; ++e) {
      if (e >= n_e) break;
      const double ze = z[e];
      const double sg = ze > 0.0 ? 1.0 : (ze < 0.0 ? -1.0 : 0.0);
      double v = -s[e] / M_PI - 0.5 * sg * X0;
      double th = occ ? (ze < 0.0 ? -1.0 : 0.0) : (ze > 0.0 ? 1.0 : 0.0);
      if (ze == 0.0) th = occ ? -0.5 : 0.5;
      if (th != 0.0) {
        const double a = fabs(ze);
        if (!(a <= top)) {   // beyond the grid, or a NaN input: no stencil index is formed
          v = NAN;
        } else {
          const double sp = a / h;
          const int i = min((int)floor(sp), n_r - 3);
          const double t = sp - i;
          const double L[4] = {-t * (t - 1.0) * (t - 2.0) / 6.0, (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0,
                               -(t + 1.0) * t * (t - 2.0) / 2.0, (t + 1.0) * t * (t - 1.0) / 6.0};
          double xv = 0.0;
#pragma unroll
          for (int o = 0; o < 4; ++o) xv += L[o] * xr[(long long)abs(i - 1 + o) * cstride];
          v += th * xv;
        }
      }
      acc[e] += v;
    }
  }
#pragma unroll
  for (int e = 0; e < CD_EMAX; ++e)
    for (int o = 32; o > 0; o >>= 1) acc[e] += __shfl_xor(acc[e], o);
  if (lane == 0)
    for (int e = 0; e < n_e; ++e) sigma_e[((long long)e * nk + k) * n_qp + n] += scale * acc[e];
}

// E[e][k][n] = e_{qp_lo+n}(k) + (e - 1) delta, e = 0, 1, 2
__global__ void k_cd_energies(const double *__restrict__ eig, int nk, int n_bands, int qp_lo, int n_qp, double delta,
                              double *__restrict__ E) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nkq = nk * n_qp;
  if (i >= 3 * nkq) return;
  const int e = i / nkq, kn = i % nkq, k = kn / n_qp, n = kn % n_qp;
  E[i] = eig[(long long)k * n_bands + qp_lo + n] + (e - 1) * delta;
}

// E_qp = e + Z (Sigma(e) + e_static), Z = 1 / (1 - (Sigma(e + d) - Sigma(e - d)) / (2 d))
__global__ void k_qp_linear(const double *__restrict__ S, const double *__restrict__ E, const double *__restrict__ e_static,
                            int nkq, double delta, double *__restrict__ e_qp, double *__restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nkq) return;
  const double Z = 1.0 / (1.0 - (S[2 * nkq + i] - S[i]) / (2.0 * delta));
  const double es = e_static ? e_static[i] : 0.0;
  e_qp[i] = E[nkq + i] + Z * (S[nkq + i] + es);
  z[i] = Z;
}

__global__ void k_count_nan(const double *__restrict__ v, int n, int *__restrict__ count) {
  __shared__ int part[256];
  int c = 0;
  for (int i = threadIdx.x; i < n; i += 256) c += isnan(v[i]) ? 1 : 0;
  part[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int i = 0; i < 256; ++i) t += part[i];
    count[0] = t;
  }
}

static int set_real_grid_broadened(lrigw_ctx *c, int n_r, double omega_max, double eta);

int run_set_real_grid(lrigw_ctx *c, int n_r, double omega_max, double eta) {
  const Dims &d = c->d;
  if (!(eta >= 0.0) || !std::isfinite(eta)) return LRIGW_ERR_ARG;
  if (eta > 0.0) return set_real_grid_broadened(c, n_r, omega_max, eta);
  if (n_r < 4 || n_r > d.n_freq || !(omega_max > 0.0) || !std::isfinite(omega_max)) return LRIGW_ERR_ARG;
  LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));   // no kernel still reads the old tables or buffers
  const double h = omega_max / (n_r - 1);
  for (int r = 0; r < d.n_freq; ++r) {
    const double w = r * h;
    c->h_om2[d.n_freq + r] = r < n_r ? -w * w : 0.0;
  }
  LRIGW_HIP_TRY(hipMemcpy(c->d_om2 + d.n_freq, c->h_om2.data() + d.n_freq, d.n_freq * sizeof(double),
                          hipMemcpyHostToDevice));
  if (n_r != c->n_real || c->real_eta > 0.0 || !c->d_chir) {
    void *bufs[] = {c->d_chir, c->d_wr, c->d_chir2, c->d_wr2, c->d_Xr};
    for (void *p : bufs)
      if (p) (void)hipFree(p);
    c->d_chir = c->d_wr = c->d_chir2 = c->d_wr2 = nullptr;
    c->d_Xr = nullptr;
    c->n_real = 0;
    const size_t plane = (size_t)d.n_aux * d.n_aux * lrigw_csize(c);
    LRIGW_HIP_TRY(hipMalloc(&c->d_chir, n_r * plane));
    LRIGW_HIP_TRY(hipMalloc(&c->d_wr, n_r * plane));
    LRIGW_HIP_TRY(hipMalloc(&c->d_chir2, n_r * plane));
    LRIGW_HIP_TRY(hipMalloc(&c->d_wr2, n_r * plane));
    LRIGW_HIP_TRY(hipMalloc(&c->d_Xr, (size_t)n_r * d.n_k * d.n_qp * d.n_bands * sizeof(double)));
  }
  if (!c->d_cdE) LRIGW_HIP_TRY(hipMalloc(&c->d_cdE, 3 * (size_t)d.n_k * d.n_qp * sizeof(double)));
  if (!c->d_cdS) LRIGW_HIP_TRY(hipMalloc(&c->d_cdS, 3 * (size_t)d.n_k * d.n_qp * sizeof(double)));
  if (!c->d_cdbad) LRIGW_HIP_TRY(hipMalloc(&c->d_cdbad, sizeof(int)));
  c->real_eta = 0.0;
  LRIGW_TRY(sigma_res_prepare_real(c, n_r));
  c->n_real = n_r;
  c->real_h = h;
  c->real_wsc_gap = -1.0;   // the FP16 scales depend on the gap: set at the next response
  return LRIGW_OK;
}

// Broadened grid: nodes w_r = r h at any height, W^c taken at w_r + i eta.
// The response of node r is built from two weight planes (Re and Im of
// 2D/(D^2 - z^2)); the pass works through the nodes in chunks of n_freq/2,
// which reuse the per-q buffers of the imaginary planes.
static int set_real_grid_broadened(lrigw_ctx *c, int n_r, double omega_max, double eta) {
  const Dims &d = c->d;
  if (n_r < 4 || n_r > 65536 || !(omega_max > 0.0) || !std::isfinite(omega_max) || d.n_freq < 2) return LRIGW_ERR_ARG;
  LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));
  void *bufs[] = {c->d_chir, c->d_wr, c->d_chir2, c->d_wr2, c->d_Xr, c->d_bom2, c->d_bcpl, c->d_bwsc};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  c->d_chir = c->d_wr = c->d_chir2 = c->d_wr2 = nullptr;
  c->d_Xr = nullptr;
  c->d_bom2 = nullptr;
  c->d_bcpl = nullptr;
  c->d_bwsc = nullptr;
  c->n_real = 0;
  const double h = omega_max / (n_r - 1);
  std::vector<double> om2(2 * (size_t)n_r);
  std::vector<double2> cpl(2 * (size_t)n_r);
  for (int r = 0; r < n_r; ++r) {
    const double w = r * h;
    om2[2 * r] = om2[2 * r + 1] = eta * eta - w * w;
    cpl[2 * r] = mkc(2.0 * w * eta, 0.0);
    cpl[2 * r + 1] = mkc(2.0 * w * eta, 1.0);
  }
  LRIGW_HIP_TRY(hipMalloc(&c->d_Xr, (size_t)n_r * d.n_k * d.n_qp * d.n_bands * sizeof(double)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_bom2, om2.size() * sizeof(double)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_bcpl, cpl.size() * sizeof(double2)));
  LRIGW_HIP_TRY(hipMalloc(&c->d_bwsc, om2.size() * sizeof(float)));
  LRIGW_HIP_TRY(hipMemcpy(c->d_bom2, om2.data(), om2.size() * sizeof(double), hipMemcpyHostToDevice));
  LRIGW_HIP_TRY(hipMemcpy(c->d_bcpl, cpl.data(), cpl.size() * sizeof(double2), hipMemcpyHostToDevice));
  c->h_bwsc.assign(om2.size(), 1.f);
  LRIGW_HIP_TRY(hipMemcpy(c->d_bwsc, c->h_bwsc.data(), c->h_bwsc.size() * sizeof(float), hipMemcpyHostToDevice));
  if (!c->d_cdE) LRIGW_HIP_TRY(hipMalloc(&c->d_cdE, 3 * (size_t)d.n_k * d.n_qp * sizeof(double)));
  if (!c->d_cdS) LRIGW_HIP_TRY(hipMalloc(&c->d_cdS, 3 * (size_t)d.n_k * d.n_qp * sizeof(double)));
  if (!c->d_cdbad) LRIGW_HIP_TRY(hipMalloc(&c->d_cdbad, sizeof(int)));
  c->sig_res_nr = 0;   // the chunks take the imaginary planes' self-energy plans or the default form
  c->sig_res_Fr = 0;
  c->sig_res_Fr4 = 0;
  c->n_real = n_r;
  c->real_h = h;
  c->real_eta = eta;
  c->bwsc_gap = c->bwsc_gmax = -1.0;
  return LRIGW_OK;
}

// FP16 split scales of the broadened planes: the largest |Re| and |Im| of
// 2D/(D^2 - z^2) over D in the transition window, sampled on 4096 log-spaced
// D plus the resonance D^2 = Re z^2, times 5/4, below 2^e
static int broadened_scales(lrigw_ctx *c) {
  if (!split_h(c->precision)) return LRIGW_OK;
  if (c->bwsc_gap == c->gap_min && c->bwsc_gmax == c->gap_max) return LRIGW_OK;
  const double lo = c->gap_min, hi = std::max(c->gap_max, c->gap_min * 1.000001), eta = c->real_eta;
  for (int r = 0; r < c->n_real; ++r) {
    const double w = r * c->real_h, p = w * w - eta * eta, sv = 2.0 * w * eta;
    double mr = 0.0, mi = 0.0;
    auto probe = [&](double D) {
      if (!(D >= lo && D <= hi)) return;
      const double a = D * D - p, den = a * a + sv * sv;
      mr = std::max(mr, std::fabs(2.0 * D * a / den));
      mi = std::max(mi, std::fabs(2.0 * D * sv / den));
    };
    for (int t = 0; t < 4096; ++t) probe(lo * std::pow(hi / lo, t / 4095.0));
    if (p > 0.0) {
      probe(std::sqrt(p));
      if (p > sv) probe(std::sqrt(p - sv));
      probe(std::sqrt(p + sv));
    }
    int e = 0;
    frexp(1.25 * std::max(mr, 1e-30), &e);
    c->h_bwsc[2 * r] = ldexpf(1.f, -e);
    frexp(1.25 * std::max(mi, 1e-30), &e);
    c->h_bwsc[2 * r + 1] = mi > 0.0 ? ldexpf(1.f, -e) : 1.f;
  }
  LRIGW_HIP_TRY(hipMemcpyAsync(c->d_bwsc, c->h_bwsc.data(), c->h_bwsc.size() * sizeof(float), hipMemcpyHostToDevice,
                               c->stream));
  LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));
  c->bwsc_gap = c->gap_min;
  c->bwsc_gmax = c->gap_max;
  return LRIGW_OK;
}

int run_chi0_real(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out) {
  const Dims &d = c->d;
  if (c->n_real < 4) return LRIGW_ERR_ARG;
  if (c->gap_trusted == 0) LRIGW_TRY(chi0_check_gap(c, eig));
  const double gap = c->gap_min;
  if (!((c->n_real - 1) * c->real_h < gap)) return LRIGW_ERR_ARG;   // a pole of the response on the grid
  if (c->real_wsc_gap != gap) {
    // FP16 split scale of plane r: the largest weight, 2D/(D^2 - w^2) at the
    // smallest D, below 2^e
    for (int r = 0; r < c->n_real; ++r) {
      const double w = r * c->real_h;
      int e = 0;
      frexp(2.0 * gap / (gap * gap - w * w), &e);
      c->h_wsc[d.n_freq + r] = ldexpf(1.f, -e);
    }
    LRIGW_HIP_TRY(hipMemcpyAsync(c->d_wsc + d.n_freq, c->h_wsc.data() + d.n_freq, c->n_real * sizeof(float),
                                 hipMemcpyHostToDevice, c->stream));
    LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));
    c->real_wsc_gap = gap;
  }
  return run_chi0_sel(c, iq, M, eig, apply_gamma, chi_out, c->d_wall, c->n_real, nullptr, true);
}

int run_sigma_cd(lrigw_ctx *c, int iq, const void *x, const void *Wc, const void *Wr, const double *eig, int n_e,
                 const double *E, double *sigma_e) {
  const Dims &d = c->d;
  if (c->n_real < 4 || n_e < 1 || n_e > CD_EMAX) return LRIGW_ERR_ARG;
  hipEvent_t ev;
  stage_begin(c, "sigma_cd", &ev);
  LRIGW_TRY(run_pair_weights(c, x, Wc, d.n_freq, (double *)c->d_X));
  LRIGW_TRY(run_pair_weights(c, x, Wr, c->n_real, c->d_Xr));
  hipLaunchKernelGGL(k_sigma_cd, dim3((unsigned)(d.n_k * d.n_qp)), dim3(64), 0, c->stream, (const double *)c->d_X, c->d_Xr,
                     eig, c->d_kmq, iq, d.n_k, d.n_qp, d.n_bands, d.n_occ, d.n_freq, c->d_omega, c->d_weight, c->n_real,
                     c->real_h, n_e, E, 1.0 / d.n_k, sigma_e);
  LRIGW_TRY(lrigw_launch_check("sigma_cd"));
  stage_end(c, "sigma_cd", ev);
  return LRIGW_OK;
}

int cd_energies(lrigw_ctx *c, const double *eig, double delta) {
  const Dims &d = c->d;
  const int n = 3 * d.n_k * d.n_qp;
  hipLaunchKernelGGL(k_cd_energies, dim3((n + 255) / 256), dim3(256), 0, c->stream, eig, d.n_k, d.n_bands, d.qp_lo, d.n_qp,
                     delta, c->d_cdE);
  return lrigw_launch_check("cd_energies");
}

int cd_qp_linear(lrigw_ctx *c, const double *S, const double *e_static, double delta, double *e_qp, double *z) {
  const Dims &d = c->d;
  const int nkq = d.n_k * d.n_qp;
  hipLaunchKernelGGL(k_qp_linear, dim3((nkq + 255) / 256), dim3(256), 0, c->stream, S, c->d_cdE, e_static, nkq, delta,
                     e_qp, z);
  return lrigw_launch_check("qp_linear");
}

int cd_count_nan(lrigw_ctx *c, const double *v, int n, int *out) {
  hipLaunchKernelGGL(k_count_nan, dim3(1), dim3(256), 0, c->stream, v, n, c->d_cdbad);
  LRIGW_TRY(lrigw_launch_check("count_nan"));
  LRIGW_HIP_TRY(hipMemcpyAsync(out, c->d_cdbad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));
  return LRIGW_OK;
}

__global__ void k_cd_set_int(int *p, int v) { p[threadIdx.x] = v; }

// Contour deformation over every q with the broadened real grid: per q the
// imaginary planes as in the exact pass, then the real nodes in chunks of
// n_freq/2 (the Re- and Im-weight responses of a chunk fill the n_freq planes
// of the second response buffer; their complex screening the second W^c
// buffer), the pair weights of each chunk into its rows of the real-grid
// array, and the combination at the n_e energy sets.  One stream; the
// screening status is folded on the device and read at the end.
int run_cd_pass_broadened(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V,
                          const void *Vcut, const void *p, double omega_cell, int n_e, const double *E, double *sigma_e,
                          int *n_bad) {
  const Dims &d = c->d;
  if (c->n_gdir > 0) return LRIGW_ERR_ARG;   // the direction average is not taken on the broadened grid
  LRIGW_TRY(driver_buffers(c));
  if (p) LRIGW_TRY(lrigw_gamma_prepare(c, V, p, omega_cell));
  LRIGW_TRY(chi0_check_gap(c, eig));
  GapScope gap_scope(c);
  LRIGW_TRY(broadened_scales(c));
  const hipStream_t s = c->stream;
  LRIGW_TRY(zero_fill(s, sigma_e, (size_t)n_e * d.n_k * d.n_qp * sizeof(double)));
  hipLaunchKernelGGL(k_cd_set_int, dim3(1), dim3(1), 0, s, c->d_info + 16, INT_MAX);
  // V(q) factors of every q at once: every chunk of real planes reuses them
  CoulombScope coulomb_scope(c);
  if (!c->capturing) LRIGW_TRY(coulomb_factors(c, V, Vcut, 0, d.n_k));
  const size_t vstride = (size_t)d.n_aux * d.n_aux;
  const long long C = (long long)d.n_k * d.n_qp * d.n_bands;
  const int P = d.n_freq / 2;
  const bool was = c->capturing;
  c->capturing = true;   // screening: device-side status, no host round trip
  int rc = LRIGW_OK;
  for (int q = 0; q < d.n_k && rc == LRIGW_OK; ++q) {
    const int g = (p && q == 0) ? 1 : 0;
    const void *Vq = (const double2 *)V + q * vstride;
    const void *Vcq = (Vcut && q > 0) ? (const void *)((const double2 *)Vcut + q * vstride) : nullptr;
    if ((rc = run_build_M(c, q, 0, H, evec, c->d_M)) < 0) break;
    if ((rc = run_chi0(c, q, c->d_M, eig, g, c->d_chi)) < 0) break;
    if ((rc = run_screen(c, q, c->d_chi, Vq, Vcq, c->d_wc, nullptr)) < 0) break;
    if ((rc = run_build_M(c, q, 1, H, evec, c->d_x)) < 0) break;
    if ((rc = run_pair_weights(c, c->d_x, c->d_wc, d.n_freq, (double *)c->d_X)) < 0) break;
    for (int r0 = 0; r0 < c->n_real && rc == LRIGW_OK; r0 += P) {
      const int np = std::min(P, c->n_real - r0);
      PlaneTab tab;
      tab.om2 = c->d_bom2 + 2 * r0;
      tab.wsc = c->d_bwsc + 2 * r0;
      tab.cpl = c->d_bcpl + 2 * r0;
      if ((rc = run_chi0_tab(c, q, c->d_M, eig, g, c->d_chi2, c->d_wall, 2 * np, nullptr, tab)) < 0) break;
      if ((rc = run_screen_cplx(c, q, c->d_chi2, Vq, Vcq, c->d_wc2, nullptr, np)) < 0) break;
      rc = run_pair_weights(c, c->d_x, c->d_wc2, np, c->d_Xr + (long long)r0 * C);
    }
    if (rc < 0) break;
    hipLaunchKernelGGL(k_sigma_cd, dim3((unsigned)(d.n_k * d.n_qp)), dim3(64), 0, s, (const double *)c->d_X, c->d_Xr,
                       eig, c->d_kmq, q, d.n_k, d.n_qp, d.n_bands, d.n_occ, d.n_freq, c->d_omega, c->d_weight, c->n_real,
                       c->real_h, n_e, E, 1.0 / d.n_k, sigma_e);
    rc = lrigw_launch_check("sigma_cd_broadened");
  }
  c->capturing = was;
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

// Newton steps on f(E) = E - e_n - e_static - Sigma^c(E).  mode 0: set the
// three energy sets E - delta, E, E + delta of the iterate (first: E = e_n);
// mode 1: E <- E + Z (e_n + e_static + S(E) - E), Z = 1/(1 - (S(E+delta) - S(E-delta))/(2 delta))
__global__ void k_cd_newton(const double *__restrict__ eig, int nk, int n_bands, int qp_lo, int n_qp,
                            const double *__restrict__ S, const double *__restrict__ e_static, double delta, int mode,
                            int first, double *__restrict__ Ecur, double *__restrict__ z, double *__restrict__ Eset) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nkq = nk * n_qp;
  if (i >= nkq) return;
  const double eps = eig[(long long)(i / n_qp) * n_bands + qp_lo + i % n_qp];
  if (mode == 0) {
    const double E = first ? eps : Ecur[i];
    if (first) Ecur[i] = eps;
    Eset[i] = E - delta;
    Eset[nkq + i] = E;
    Eset[2 * nkq + i] = E + delta;
    return;
  }
  const double E = Ecur[i];
  const double Z = 1.0 / (1.0 - (S[2 * nkq + i] - S[i]) / (2.0 * delta));
  Ecur[i] = E + Z * (eps + (e_static ? e_static[i] : 0.0) + S[nkq + i] - E);
  if (z) z[i] = Z;
}

int cd_newton(lrigw_ctx *c, const double *eig, const double *S, const double *e_static, double delta, double *e_cur,
              double *z, int first) {
  const Dims &d = c->d;
  const int nkq = d.n_k * d.n_qp;
  hipLaunchKernelGGL(k_cd_newton, dim3((nkq + 255) / 256), dim3(256), 0, c->stream, eig, d.n_k, d.n_bands, d.qp_lo, d.n_qp,
                     S, e_static, delta, S ? 1 : 0, first, e_cur, z, c->d_cdE);
  return lrigw_launch_check("cd_newton");
}
