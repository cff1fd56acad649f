// Analytic continuation of Sigma^c(i w) (Thiele continued fraction, Vidberg and
// Serene 1977) and the quasiparticle equation, FP64, one thread per (k, n).
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

#define NPMAX 64
#define PADE_TINY 1e-300

__device__ inline double2 zdiv(double2 a, double2 b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return mkc((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  }
  double r = b.x / b.y, den = b.x * r + b.y;
  return mkc((a.x * r + a.y) / den, (a.y * r - a.x) / den);
}
__device__ inline bool zfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }
__device__ inline double zabs(double2 a) { return hypot(a.x, a.y); }

// value and derivative of the continued fraction at real z
__device__ inline void cf_eval(const double2 *a, const double2 *zn, int na, double z, double2 &val, double2 &der) {
  if (na == 0) {
    val = mkc(0.0, 0.0);
    der = mkc(0.0, 0.0);
    return;
  }
  double2 A0 = mkc(0.0, 0.0), A1 = a[0], B0 = mkc(1.0, 0.0), B1 = mkc(1.0, 0.0);
  double2 dA0 = mkc(0.0, 0.0), dA1 = mkc(0.0, 0.0), dB0 = mkc(0.0, 0.0), dB1 = mkc(0.0, 0.0);
  for (int p = 1; p < na; ++p) {
    double2 zz = mkc(z - zn[p - 1].x, -zn[p - 1].y);
    double2 t = cmul(a[p], zz);
    double2 A2 = cadd(A1, cmul(t, A0));
    double2 B2 = cadd(B1, cmul(t, B0));
    double2 dA2 = cadd(cadd(dA1, cmul(a[p], A0)), cmul(t, dA0));
    double2 dB2 = cadd(cadd(dB1, cmul(a[p], B0)), cmul(t, dB0));
    A0 = A1; A1 = A2; B0 = B1; B1 = B2;
    dA0 = dA1; dA1 = dA2; dB0 = dB1; dB1 = dB2;
  }
  val = zdiv(A1, B1);
  double2 num = mkc(dA1.x * B1.x - dA1.y * B1.y - (A1.x * dB1.x - A1.y * dB1.y),
                    dA1.x * B1.y + dA1.y * B1.x - (A1.x * dB1.y + A1.y * dB1.x));
  der = zdiv(num, cmul(B1, B1));
}

// nodes z_j = i w_node(j) (n_par grid points j (n_freq-1)/(n_par-1), rounded
// half up) and the continued-fraction coefficients of one (k, n) row of
// sigma, by inverse differences; returns the number of coefficients kept
// (the fraction is truncated at a zero or non-finite one)
__device__ inline int pade_coeffs(const double2 *__restrict__ row, int n_freq, int n_par, const double *__restrict__ omega,
                                  double2 *zn, double2 *a) {
  double2 g[NPMAX];
  for (int j = 0; j < n_par; ++j) {
    int node = (n_par == 1) ? 0 : (int)((2LL * j * (n_freq - 1) + (n_par - 1)) / (2LL * (n_par - 1)));
    zn[j] = mkc(0.0, omega[node]);
    g[j] = row[node];
  }
  int na = n_par;
  a[0] = g[0];
  if (!(zfinite(a[0]) && zabs(a[0]) >= PADE_TINY)) return 0;
  for (int p = 1; p < n_par; ++p) {
    for (int j = n_par - 1; j >= p; --j) {
      double2 num = mkc(g[p - 1].x - g[j].x, g[p - 1].y - g[j].y);
      double2 den = cmul(mkc(zn[j].x - zn[p - 1].x, zn[j].y - zn[p - 1].y), g[j]);
      g[j] = zdiv(num, den);
    }
    a[p] = g[p];
    if (!zfinite(a[p]) || zabs(a[p]) < PADE_TINY) {
      na = p;
      break;
    }
  }
  return na;
}

// P(E - mu) at n_e sets of real energies: out[e][k][n] = P_{kn}(E[e][k][n] - mu)
__global__ void k_pade_eval(const double2 *__restrict__ sigma, int nkq, int n_freq, int n_par,
                            const double *__restrict__ omega, double mu, int n_e, const double *__restrict__ E,
                            double2 *__restrict__ out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nkq) return;
  double2 zn[NPMAX], a[NPMAX];
  const int na = pade_coeffs(sigma + (long long)idx * n_freq, n_freq, n_par, omega, zn, a);
  for (int e = 0; e < n_e; ++e) {
    double2 v, dv;
    cf_eval(a, zn, na, E[(long long)e * nkq + idx] - mu, v, dv);
    out[(long long)e * nkq + idx] = v;
  }
}

__global__ void k_pade_qp(const double2 *__restrict__ sigma, int nkq, int n_freq, int n_par, const double *__restrict__ omega,
                          const double *__restrict__ eps_qp, const double *__restrict__ e_static, double mu,
                          double *__restrict__ e_qp, double *__restrict__ zf, int *__restrict__ flags) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nkq) return;
  double2 zn[NPMAX], a[NPMAX];
  const int na = pade_coeffs(sigma + (long long)idx * n_freq, n_freq, n_par, omega, zn, a);
  if (na < n_par) atomicAdd(flags + 1, 1);
  const double target = eps_qp[idx] + (e_static ? e_static[idx] : 0.0);
  double2 v, dv;
  double E = target;
  bool ok = false;
  double Z = 1.0;
  // Newton, abandoned once f' <= 0 (the iterate crossed a pole of the fraction)
  for (int it = 0; it < 50; ++it) {
    cf_eval(a, zn, na, E - mu, v, dv);
    double fv = E - target - v.x, fd = 1.0 - dv.x;
    if (!(isfinite(fv) && isfinite(fd)) || fd <= 0.0) break;
    double dE = fv / fd;
    E -= dE;
    if (fabs(dE) < 1e-10) {
      cf_eval(a, zn, na, E - mu, v, dv);
      if (1.0 - dv.x > 0.0) {
        Z = 1.0 / (1.0 - dv.x);
        ok = true;
      }
      break;
    }
  }
  if (!ok) {
    // scan E0 +- 1 Ha in 1 mHa steps for increasing sign changes (roots, not
    // poles), bracket nearest to the start, bisection
    int best = 0;
    bool found = false;
    double bestd = 0.0, fprev = 0.0;
    for (int i = -1000; i <= 1000; ++i) {
      double x = target + i * 1e-3;
      cf_eval(a, zn, na, x - mu, v, dv);
      double f = x - target - v.x;
      if (i > -1000) {
        double xp = target + (i - 1) * 1e-3;
        if (isfinite(fprev) && isfinite(f) && fprev < 0.0 && f >= 0.0) {
          double mid = 0.5 * (xp + x);
          double dd = fabs(mid - target);
          if (!found || dd < bestd) {
            best = i - 1;
            bestd = dd;
            found = true;
          }
        }
      }
      fprev = f;
    }
    if (!found) {
      cf_eval(a, zn, na, target - mu, v, dv);
      E = target;
      Z = 1.0 / (1.0 - dv.x);
      atomicAdd(flags + 0, 1);
    } else {
      double lo = target + best * 1e-3, hi = target + (best + 1) * 1e-3;
      for (int it = 0; it < 200; ++it) {
        if (hi - lo < 1e-12) break;
        double mid = 0.5 * (lo + hi);
        cf_eval(a, zn, na, mid - mu, v, dv);
        double fm = mid - target - v.x;
        if (fm >= 0.0) hi = mid;
        else lo = mid;
      }
      E = 0.5 * (lo + hi);
      cf_eval(a, zn, na, E - mu, v, dv);
      Z = 1.0 / (1.0 - dv.x);
    }
  }
  e_qp[idx] = E;
  zf[idx] = Z;
}

__global__ void k_flags_init(int *f) { f[threadIdx.x] = 0; }

int run_qp(lrigw_ctx *c, const void *sigma, const double *eps_qp, const double *e_static, int n_par, double *e_qp, double *z,
           int *info) {
  const Dims &d = c->d;
  if (n_par > d.n_freq) n_par = d.n_freq;
  if (n_par > NPMAX) return LRIGW_ERR_ARG;
  int nkq = d.n_k * d.n_qp;
  int *flags = c->d_info + 8;
  hipLaunchKernelGGL(k_flags_init, dim3(1), dim3(2), 0, c->stream, flags);
  hipLaunchKernelGGL(k_pade_qp, dim3((nkq + 63) / 64), dim3(64), 0, c->stream, (const double2 *)sigma, nkq, d.n_freq, n_par,
                     c->d_omega, eps_qp, e_static, d.mu, e_qp, z, flags);
  LRIGW_TRY(lrigw_launch_check("pade_qp"));
  if (c->capturing) {   // flags stay in d_info[8..9]
    if (info) *info = 0;
    return LRIGW_OK;
  }
  int h[2];
  LRIGW_HIP_TRY(hipMemcpyAsync(h, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));
  if (info) *info = h[0];
  if (h[0] > 0) return LRIGW_WARN_QP_NOCONV;
  if (h[1] > 0) return LRIGW_WARN_PADE_TRUNC;
  return LRIGW_OK;
}

int run_pade_eval(lrigw_ctx *c, const void *sigma, int n_par, int n_e, const double *E, void *out) {
  const Dims &d = c->d;
  if (n_par > d.n_freq) n_par = d.n_freq;
  if (n_par < 1 || n_par > NPMAX) return LRIGW_ERR_ARG;
  const int nkq = d.n_k * d.n_qp;
  hipLaunchKernelGGL(k_pade_eval, dim3((nkq + 63) / 64), dim3(64), 0, c->stream, (const double2 *)sigma, nkq, d.n_freq, n_par,
                     c->d_omega, d.mu, n_e, E, (double2 *)out);
  return lrigw_launch_check("pade_eval");
}

