// Learned frequency surrogate of the response (the learned form; not in the
// paper, which evaluates Eq. chi0_matrix at every grid frequency).
//
// Per q the response is computed exactly at n_a anchor frequencies and one
// held-out frequency.  Everywhere else it is predicted as
//   chi(w_t) = sum_l c_l(w_t) chi(w_l) + U R_t U^H,
// with c(w) a least-squares interpolation rule fitted to the transition
// kernel 2D/(D^2 + w^2) over the transition-energy window, U an orthonormal
// basis of the dominant eigenspace of -chi(w_a0) (subspace iteration, Cholesky
// QR), and R_t the residual of the rule on the r x r projection U^H chi U,
// predicted per real series (Re above and on the diagonal, Im below) by a
// three-layer tanh network from the series' scaled anchor values.  If the
// relative Frobenius error of the prediction at the held-out frequency exceeds
// a threshold, the exact kernels recompute every other frequency of this q
// (a device flag: no host round trip).
//
// Network: BF16 weights (FP32 master copy for Adam), FP32 activations, FP32
// MFMA 16x16x4 products with FP32 accumulation.  Each affine layer is one GEMM
// with the bias folded in as an extra row of the weight matrix (a constant-one
// column of the activations), so the flat parameter vector is the three
// augmented weight matrices back to back.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "lrigw_internal.h"
#include "tiles.h"

struct lrigw_surrogate {
  int n_aux = 0, n_freq = 0, rank = 0, n_anchor = 0, hidden = 0, n_out = 0, n_iter = 4;
  double x0 = 0.0, d_lo = 0.0, d_hi = 0.0;
  int holdout = 0, t_holdout = 0;
  std::vector<int> anchors, targets;
  hipStream_t stream = nullptr;
  // tables
  double *d_C = nullptr;         // [n_a][n_out] rule weights
  int *d_asel = nullptr;         // anchors then the held-out index (n_a + 1)
  int *d_tall = nullptr;         // every non-anchor index (n_out)
  int *d_trest = nullptr;        // non-anchor indices except the held-out one (n_out - 1)
  double2 *d_start = nullptr;    // [N][r]
  double2 *d_U = nullptr, *d_Y = nullptr;      // [N][r]
  double2 *d_G = nullptr, *d_Linv = nullptr;   // [r][r]
  double2 *d_dinv = nullptr;
  double2 *d_T = nullptr;        // [n_freq][N][r]
  double2 *d_P = nullptr;        // [n_freq][r][r]
  double2 *d_R = nullptr;        // [n_out][r][r]
  int *d_info = nullptr;         // [4]
  // network
  long long n_par = 0, o2 = 0, o3 = 0;
  float *d_theta = nullptr, *d_m = nullptr, *d_v = nullptr, *d_grad = nullptr;
  uint16_t *d_wb = nullptr;      // BF16 weights used by the products
  long long adam_t = 0;
  // batch buffers
  int bcap = 0;
  float *d_xb = nullptr, *d_yb = nullptr, *d_h1 = nullptr, *d_h2 = nullptr, *d_dz1 = nullptr, *d_dz2 = nullptr;
  float *d_dy = nullptr, *d_part = nullptr, *d_loss_part = nullptr;
  double *d_sig = nullptr;
  long long part_cap = 0;
  // training rows
  long long row_cap = 0, n_rows = 0;
  float *d_xdata = nullptr, *d_ydata = nullptr;
  // fallback bookkeeping
  int *d_run = nullptr;          // 1: recompute exactly
  int *d_nfb = nullptr;          // number of fallbacks
  double *d_err = nullptr;       // held-out errors, one per call (cyclic, ERR_LOG)
  double *d_nmax = nullptr;      // largest series norm of the current q
  long long n_calls = 0;
};

#define ERR_LOG 65536

// ---------------------------------------------------------------- host: interpolation rule
// Least squares by Householder QR: minimise |A x - b|, A m x n (m >= n), column-major.
static void lsq_householder(std::vector<double> A, int m, int n, std::vector<double> b, double *x) {
  for (int j = 0; j < n; ++j) {
    double nrm = 0.0;
    for (int i = j; i < m; ++i) nrm += A[(size_t)j * m + i] * A[(size_t)j * m + i];
    nrm = std::sqrt(nrm);
    const double a0 = A[(size_t)j * m + j];
    const double alpha = a0 > 0 ? -nrm : nrm;
    std::vector<double> v(m, 0.0);
    for (int i = j; i < m; ++i) v[i] = A[(size_t)j * m + i];
    v[j] -= alpha;
    double vv = 0.0;
    for (int i = j; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int c = j; c < n; ++c) {
      double s = 0.0;
      for (int i = j; i < m; ++i) s += v[i] * A[(size_t)c * m + i];
      s = 2.0 * s / vv;
      for (int i = j; i < m; ++i) A[(size_t)c * m + i] -= s * v[i];
    }
    double s = 0.0;
    for (int i = j; i < m; ++i) s += v[i] * b[i];
    s = 2.0 * s / vv;
    for (int i = j; i < m; ++i) b[i] -= s * v[i];
  }
  for (int j = n - 1; j >= 0; --j) {
    double s = b[j];
    for (int c = j + 1; c < n; ++c) s -= A[(size_t)c * m + j] * x[c];
    x[j] = s / A[(size_t)j * m + j];
  }
}

static double gker(double D, double w) { return 2.0 * D / (D * D + w * w); }

// c[l][t]: the anchor columns of G = [g_D(w_l)] over a log-spaced family of D
// are scaled to unit norm n_l, [G/n; sqrt(ridge) I] c' = [g_D(w_t); 0] is
// solved in the least-squares sense and c_l = c'_l / n_l.
static void rule_weights(const std::vector<double> &omega, const std::vector<int> &anchors,
                         const std::vector<int> &targets, double d_lo, double d_hi, std::vector<double> &C) {
  const int nd = 256, na = (int)anchors.size(), nt = (int)targets.size();
  const double ridge = 1e-12;
  std::vector<double> D(nd);
  for (int i = 0; i < nd; ++i) D[i] = d_lo * std::pow(d_hi / d_lo, i / (nd - 1.0));
  std::vector<double> nrm(na, 0.0);
  for (int l = 0; l < na; ++l) {
    for (int i = 0; i < nd; ++i) nrm[l] += gker(D[i], omega[anchors[l]]) * gker(D[i], omega[anchors[l]]);
    nrm[l] = std::sqrt(nrm[l]);
  }
  const int m = nd + na;
  std::vector<double> A((size_t)m * na, 0.0);
  for (int l = 0; l < na; ++l) {
    for (int i = 0; i < nd; ++i) A[(size_t)l * m + i] = gker(D[i], omega[anchors[l]]) / nrm[l];
    A[(size_t)l * m + nd + l] = std::sqrt(ridge);
  }
  C.assign((size_t)na * nt, 0.0);
  std::vector<double> x(na);
  for (int t = 0; t < nt; ++t) {
    std::vector<double> b(m, 0.0);
    for (int i = 0; i < nd; ++i) b[i] = gker(D[i], omega[targets[t]]);
    lsq_householder(A, m, na, b, x.data());
    for (int l = 0; l < na; ++l) C[(size_t)l * nt + t] = x[l] / nrm[l];
  }
}

// ---------------------------------------------------------------- network GEMM (FP32 MFMA)
// P[z] = sum_{k in chunk z} A(m,k) B(k,n) for an M x N output; A(m,k) = A[m][k]
// (a_t = 0) or A[k][m] (a_t = 1), with a constant one at k == a_aug (a_t = 0)
// or m == a_aug (a_t = 1); B(k,n) = B[k][n] (b_t = 0) or B[n][k] (b_t = 1),
// FP32 or BF16 storage.
struct MG {
  int M, N, K;
  const float *A;
  long long lda;
  int a_t, a_aug;
  const void *B;
  long long ldb;
  int b_t, b_bf16;
  float *P;
  long long kchunk;
};

#define MKC 16
#define MLP 68

__device__ inline float bf16_to_f(uint16_t u) { return __uint_as_float(((uint32_t)u) << 16); }

__global__ __launch_bounds__(256) void k_mlp_gemm(MG g) {
  __shared__ float As[MKC][MLP];
  __shared__ float Bs[MKC][MLP];
  const int m0 = blockIdx.y * TILE, n0 = blockIdx.x * TILE;
  const long long kb = (long long)blockIdx.z * g.kchunk;
  const long long ke = min((long long)g.K, kb + g.kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, col = lane & 15;
  f4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<float>::zero();
  for (long long k0 = kb; k0 < ke; k0 += MKC) {
#pragma unroll
    for (int t = 0; t < (MKC * TILE) / 256; ++t) {
      const int e = tid + 256 * t;
      int mm, kk;
      if (g.a_t == 0) { mm = e / MKC; kk = e % MKC; } else { kk = e / TILE; mm = e % TILE; }
      const int m = m0 + mm;
      const long long k = k0 + kk;
      float v = 0.f;
      if (m < g.M && k < ke) {
        if (g.a_t == 0) v = (k == g.a_aug) ? 1.f : g.A[(long long)m * g.lda + k];
        else v = (m == g.a_aug) ? 1.f : g.A[k * g.lda + m];
      }
      As[kk][mm] = v;
      int nn;
      if (g.b_t == 0) { kk = e / TILE; nn = e % TILE; } else { nn = e / MKC; kk = e % MKC; }
      const int n = n0 + nn;
      const long long kq = k0 + kk;
      float u = 0.f;
      if (n < g.N && kq < ke) {
        const long long off = g.b_t == 0 ? kq * g.ldb + n : (long long)n * g.ldb + kq;
        u = g.b_bf16 ? bf16_to_f(((const uint16_t *)g.B)[off]) : ((const float *)g.B)[off];
      }
      Bs[kk][nn] = u;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < MKC / 4; ++ks) {
      const int kk = 4 * ks + (lane >> 4);
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[kk][32 * wr + 16 * i + col];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk][32 * wc + 16 * j + col];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<float>::mac(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  float *P = g.P + (long long)blockIdx.z * g.M * g.N;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + 32 * wr + 16 * i + Mfma<float>::row(lane, r);
        const int cc = n0 + 32 * wc + 16 * j + col;
        if (row < g.M && cc < g.N) P[(long long)row * g.N + cc] = acc[i][j][r];
      }
}

static int mlp_gemm(hipStream_t s, const MG &g0) {
  MG g = g0;
  if (g.kchunk <= 0) g.kchunk = g.K;
  const long long S = (g.K + g.kchunk - 1) / g.kchunk;
  dim3 grid((unsigned)((g.N + TILE - 1) / TILE), (unsigned)((g.M + TILE - 1) / TILE), (unsigned)S);
  hipLaunchKernelGGL(k_mlp_gemm, grid, dim3(256), 0, s, g);
  return lrigw_launch_check("mlp_gemm");
}

__global__ void k_mlp_tanh(const float *__restrict__ P, long long n, float *__restrict__ h) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) h[i] = tanhf(P[i]);
}

// dz = P (1 - h^2)
__global__ void k_mlp_dtanh(const float *__restrict__ P, const float *__restrict__ h, long long n, float *__restrict__ dz) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dz[i] = P[i] * (1.f - h[i] * h[i]);
}

// dY = scale (y - target); per-block partial sums of (y - target)^2
__global__ void k_mlp_out(const float *__restrict__ y, const float *__restrict__ tgt, long long n, float scale,
                          float *__restrict__ dy, float *__restrict__ loss_part) {
  __shared__ float red[256];
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  float d = 0.f;
  if (i < n) {
    d = y[i] - tgt[i];
    dy[i] = scale * d;
  }
  red[threadIdx.x] = d * d;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

__global__ void k_loss_sum(const float *__restrict__ part, int n, double inv, float *__restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += (double)part[i];
  out[0] = (float)(s * inv);
}

// out[i] = sum_z P[z][i] (fixed order)
__global__ void k_sum_parts(const float *__restrict__ P, int S, long long n, float *__restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int z = 0; z < S; ++z) s += P[(long long)z * n + i];
  out[i] = s;
}

__device__ inline uint16_t f_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void k_adam(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ g,
                       long long n, float lr, float b1, float b2, float eps, float c1, float c2, uint16_t *__restrict__ wb) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float t = th[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  th[i] = t;
  wb[i] = f_to_bf16(t);
}

__global__ void k_to_bf16(const float *__restrict__ th, long long n, uint16_t *__restrict__ wb) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wb[i] = f_to_bf16(th[i]);
}

__global__ void k_gather_rows(const float *__restrict__ xd, const float *__restrict__ yd, const int *__restrict__ order,
                              long long off, int B, int n_in, int n_out, long long n_rows, float *__restrict__ xb,
                              float *__restrict__ yb) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = n_in + n_out;
  if (i >= (long long)B * w) return;
  const int b = (int)(i / w), c = (int)(i % w);
  long long r = order[off + b];
  r = r < 0 ? 0 : (r >= n_rows ? n_rows - 1 : r);
  if (c < n_in) xb[(long long)b * n_in + c] = xd[r * n_in + c];
  else yb[(long long)b * n_out + (c - n_in)] = yd[r * n_out + (c - n_in)];
}

// ---------------------------------------------------------------- series kernels
__device__ inline double series_val(const double2 *P, int r, int s) {
  const int i = s / r, j = s % r;
  const double2 v = P[(long long)i * r + j];
  return i <= j ? v.x : v.y;
}

// Series whose anchor norm is at most NOISE_FLOOR times the largest one of
// the q have no shape above rounding (e.g. imaginary parts at a time-reversal
// invariant q): scale 0, features 0, targets 0.
#define NOISE_FLOOR 1e-6

// largest anchor norm over the r^2 series (one workgroup); asel == nullptr:
// anchors are P[0..n_a-1]
__global__ __launch_bounds__(1024) void k_series_norm_max(const double2 *__restrict__ P, int r, const int *__restrict__ asel,
                                                          int n_a, double *__restrict__ out) {
  __shared__ double red[1024];
  double m = 0.0;
  for (int s = threadIdx.x; s < r * r; s += blockDim.x) {
    double nrm = 0.0;
    for (int l = 0; l < n_a; ++l) {
      const double v = series_val(P + (long long)(asel ? asel[l] : l) * r * r, r, s);
      nrm += v * v;
    }
    m = fmax(m, sqrt(nrm));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// training rows of every series: anchors -> x, rule residual at the targets -> y
__global__ void k_series_rows(const double2 *__restrict__ P, int r, const int *__restrict__ asel, int n_a,
                              const int *__restrict__ tall, int n_out, const double *__restrict__ C,
                              const double *__restrict__ nmax, float *__restrict__ xo, float *__restrict__ yo) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= r * r) return;
  double a[16];
  double nrm = 0.0;
  for (int l = 0; l < n_a; ++l) {
    a[l] = series_val(P + (long long)asel[l] * r * r, r, s);
    nrm += a[l] * a[l];
  }
  nrm = sqrt(nrm);
  if (!(nrm > NOISE_FLOOR * nmax[0])) nrm = 0.0;
  const double sg = a[0] < 0.0 ? -nrm : nrm;
  const double inv = sg != 0.0 ? 1.0 / sg : 0.0;
  for (int l = 0; l < n_a; ++l) xo[(long long)s * n_a + l] = (float)(a[l] * inv);
  for (int t = 0; t < n_out; ++t) {
    double base = 0.0;
    for (int l = 0; l < n_a; ++l) base += C[(long long)l * n_out + t] * a[l];
    const double f = series_val(P + (long long)tall[t] * r * r, r, s);
    yo[(long long)s * n_out + t] = (float)((f - base) * inv);
  }
}

// inference features from the anchor projections P[l] (l = 0..n_a-1, contiguous)
__global__ void k_series_features(const double2 *__restrict__ P, int r, int n_a, const double *__restrict__ nmax,
                                  float *__restrict__ xo, double *__restrict__ sig) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= r * r) return;
  double a[16];
  double nrm = 0.0;
  for (int l = 0; l < n_a; ++l) {
    a[l] = series_val(P + (long long)l * r * r, r, s);
    nrm += a[l] * a[l];
  }
  nrm = sqrt(nrm);
  if (!(nrm > NOISE_FLOOR * nmax[0])) nrm = 0.0;
  const double sg = a[0] < 0.0 ? -nrm : nrm;
  const double inv = sg != 0.0 ? 1.0 / sg : 0.0;
  for (int l = 0; l < n_a; ++l) xo[(long long)s * n_a + l] = (float)(a[l] * inv);
  sig[s] = sg;
}

// R[t] (Hermitian r x r) from the predicted residual series y[s][t] * sig[s]
__global__ void k_series_residual(const float *__restrict__ y, const double *__restrict__ sig, int r, int n_out,
                                  double2 *__restrict__ R) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long rr = (long long)r * r;
  if (idx >= rr * n_out) return;
  const int t = (int)(idx / rr);
  const int i = (int)((idx % rr) / r), j = (int)(idx % r);
  auto S = [&](int a, int b) { const int s = a * r + b; return (double)y[(long long)s * n_out + t] * sig[s]; };
  double2 v;
  if (i == j) v = mkc(S(i, i), 0.0);
  else if (i < j) v = mkc(S(i, j), -S(j, i));
  else v = mkc(S(j, i), S(i, j));
  R[idx] = v;
}

template <typename T>
__global__ void k_widen_sel(const typename c2t<T>::type *__restrict__ chi, const int *__restrict__ sel, long long nn,
                            double2 *__restrict__ out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nn) return;
  out[(long long)blockIdx.y * nn + i] = to_z(chi[(long long)sel[blockIdx.y] * nn + i]);
}

// chi(w_t) = sum_l C[l][t] chi_a[l] + T2[t]; the held-out target goes to `hold`
template <typename T>
__global__ void k_sur_combine(const double2 *__restrict__ chia, int n_a, const double *__restrict__ C, int n_out,
                              const double2 *__restrict__ T2, const int *__restrict__ tall, int t_hold, long long nn,
                              typename c2t<T>::type *__restrict__ chi, double2 *__restrict__ hold) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int t = blockIdx.y;
  if (i >= nn) return;
  double2 v = T2[(long long)t * nn + i];
  for (int l = 0; l < n_a; ++l) {
    const double c = C[(long long)l * n_out + t];
    const double2 a = chia[(long long)l * nn + i];
    v.x += c * a.x;
    v.y += c * a.y;
  }
  if (t == t_hold) hold[i] = v;
  else chi[(long long)tall[t] * nn + i] = to_c<T>(v);
}

// relative Frobenius error at the held-out frequency; run = error > threshold
// (or not finite); one workgroup
__global__ __launch_bounds__(1024) void k_sur_check(const double2 *__restrict__ pred, const double2 *__restrict__ exact,
                                                    long long nn, double thr, int *__restrict__ run, int *__restrict__ nfb,
                                                    double *__restrict__ err_log, long long slot) {
  __shared__ double rn[1024], rd[1024];
  double sn = 0.0, sd = 0.0;
  for (long long i = threadIdx.x; i < nn; i += blockDim.x) {
    const double2 p = pred[i], e = exact[i];
    const double dx = p.x - e.x, dy = p.y - e.y;
    sn += dx * dx + dy * dy;
    sd += e.x * e.x + e.y * e.y;
  }
  rn[threadIdx.x] = sn;
  rd[threadIdx.x] = sd;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      rn[threadIdx.x] += rn[threadIdx.x + st];
      rd[threadIdx.x] += rd[threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e = rd[0] > 0.0 ? sqrt(rn[0] / rd[0]) : (rn[0] > 0.0 ? INFINITY : 0.0);
    const int fb = (e <= thr) ? 0 : 1;   // NaN compares false -> fallback
    run[0] = fb;
    nfb[0] += fb;
    err_log[slot % ERR_LOG] = e;
  }
}

__global__ void k_set_identity(double2 *A, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) A[i] = mkc((i / n == i % n) ? 1.0 : 0.0, 0.0);
}

__global__ void k_real_to_z(const double *__restrict__ a, long long n, double2 *__restrict__ z) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = mkc(a[i], 0.0);
}

__global__ void k_zero_int(int *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// ---------------------------------------------------------------- host helpers
static ZGemm zg(int m, int n, int k, int opa, const double2 *A, long long lda, long long sa, int opb, const double2 *B,
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

static unsigned nblk(long long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// U = orthonormal basis of span((-chi)^n_iter start): Cholesky QR after every product.
// chi0: FP64 [N][N] on the device.  d_info[0] != INT_MAX after a failed Cholesky.
static int sur_basis(lrigw_surrogate *sg, hipStream_t s, const double2 *chi0) {
  const int N = sg->n_aux, r = sg->rank;
  const double2 one = mkc(1.0, 0.0), mone = mkc(-1.0, 0.0);
  const double2 *Q = sg->d_start;
  for (int it = 0; it < sg->n_iter; ++it) {
    LRIGW_TRY(zgemm(s, zg(N, r, N, OP_N, chi0, N, 0, OP_N, Q, r, 0, sg->d_Y, r, 0, mone, 1)));
    LRIGW_TRY(zgemm(s, zg(r, r, N, OP_C, sg->d_Y, r, 0, OP_N, sg->d_Y, r, 0, sg->d_G, r, 0, one, 1)));
    LRIGW_TRY(zpotrf_batched(s, sg->d_G, r, r, (long long)r * r, 1, sg->d_dinv, sg->d_info + it % 2));
    hipLaunchKernelGGL(k_set_identity, dim3(nblk((long long)r * r)), dim3(256), 0, s, sg->d_Linv, r);
    LRIGW_TRY(ztrsm_left_lower(s, sg->d_G, r, 0, sg->d_dinv, sg->d_Linv, r, 0, r, r, 1));
    LRIGW_TRY(zgemm(s, zg(N, r, r, OP_N, sg->d_Y, r, 0, OP_C, sg->d_Linv, r, 0, sg->d_U, r, 0, one, 1)));
    Q = sg->d_U;
  }
  return lrigw_launch_check("surrogate_basis");
}

// P[w] = U^H chi[w] U for nw FP64 matrices
static int sur_project(lrigw_surrogate *sg, hipStream_t s, const double2 *chi, int nw) {
  const int N = sg->n_aux, r = sg->rank;
  const long long nn = (long long)N * N;
  const double2 one = mkc(1.0, 0.0);
  LRIGW_TRY(zgemm(s, zg(N, r, N, OP_N, chi, N, nn, OP_N, sg->d_U, r, 0, sg->d_T, r, (long long)N * r, one, nw)));
  LRIGW_TRY(zgemm(s, zg(r, r, N, OP_C, sg->d_U, r, 0, OP_N, sg->d_T, r, (long long)N * r, sg->d_P, r, (long long)r * r, one,
                        nw)));
  return LRIGW_OK;
}

static int ensure_batch(lrigw_surrogate *sg, int B) {
  if (B <= sg->bcap) return LRIGW_OK;
  float **fl[] = {&sg->d_xb, &sg->d_yb, &sg->d_h1, &sg->d_h2, &sg->d_dz1, &sg->d_dz2, &sg->d_dy, &sg->d_part, &sg->d_loss_part};
  for (float **p : fl)
    if (*p) { (void)hipFree(*p); *p = nullptr; }
  if (sg->d_sig) { (void)hipFree(sg->d_sig); sg->d_sig = nullptr; }
  const int H = sg->hidden, no = sg->n_out, ni = sg->n_anchor;
  const int W = std::max(H, no);
  const long long S = (B + 255) / 256;
  sg->part_cap = std::max<long long>((long long)B * W, S * (long long)(H + 1) * W);
  LRIGW_HIP_TRY(hipMalloc(&sg->d_xb, (size_t)B * ni * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_yb, (size_t)B * no * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_h1, (size_t)B * H * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_h2, (size_t)B * H * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_dz1, (size_t)B * H * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_dz2, (size_t)B * H * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_dy, (size_t)B * no * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_part, (size_t)sg->part_cap * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_loss_part, (size_t)nblk((long long)B * no) * sizeof(float)));
  LRIGW_HIP_TRY(hipMalloc(&sg->d_sig, (size_t)B * sizeof(double)));
  sg->bcap = B;
  return LRIGW_OK;
}

// forward pass of B rows x [B][n_in]; leaves h1, h2 and y (= d_part, [B][n_out])
static int mlp_forward(lrigw_surrogate *sg, hipStream_t s, const float *x, int B) {
  const int H = sg->hidden, no = sg->n_out, ni = sg->n_anchor;
  MG g;
  g = {B, H, ni + 1, x, ni, 0, ni, sg->d_wb, H, 0, 1, sg->d_part, 0};
  LRIGW_TRY(mlp_gemm(s, g));
  hipLaunchKernelGGL(k_mlp_tanh, dim3(nblk((long long)B * H)), dim3(256), 0, s, sg->d_part, (long long)B * H, sg->d_h1);
  g = {B, H, H + 1, sg->d_h1, H, 0, H, sg->d_wb + sg->o2, H, 0, 1, sg->d_part, 0};
  LRIGW_TRY(mlp_gemm(s, g));
  hipLaunchKernelGGL(k_mlp_tanh, dim3(nblk((long long)B * H)), dim3(256), 0, s, sg->d_part, (long long)B * H, sg->d_h2);
  g = {B, no, H + 1, sg->d_h2, H, 0, H, sg->d_wb + sg->o3, no, 0, 1, sg->d_part, 0};
  LRIGW_TRY(mlp_gemm(s, g));
  return lrigw_launch_check("mlp_forward");
}

// loss and gradient (into d_grad) of the rows xb, yb; loss -> loss_out[0] (device)
static int mlp_grad(lrigw_surrogate *sg, hipStream_t s, const float *xb, const float *yb, int B, float *loss_out) {
  const int H = sg->hidden, no = sg->n_out, ni = sg->n_anchor;
  LRIGW_TRY(mlp_forward(sg, s, xb, B));
  const long long ny = (long long)B * no;
  hipLaunchKernelGGL(k_mlp_out, dim3(nblk(ny)), dim3(256), 0, s, sg->d_part, yb, ny, (float)(2.0 / (double)ny), sg->d_dy,
                     sg->d_loss_part);
  hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(1), 0, s, sg->d_loss_part, (int)nblk(ny), 1.0 / (double)ny, loss_out);
  const long long kc = 256;
  const int S = (int)((B + kc - 1) / kc);
  MG g;
  // gW3 = [h2 1]^T dY
  g = {H + 1, no, B, sg->d_h2, H, 1, H, sg->d_dy, no, 0, 0, sg->d_part, kc};
  LRIGW_TRY(mlp_gemm(s, g));
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk((long long)(H + 1) * no)), dim3(256), 0, s, sg->d_part, S,
                     (long long)(H + 1) * no, sg->d_grad + sg->o3);
  // dz2 = (dY W3^T) (1 - h2^2)
  g = {B, H, no, sg->d_dy, no, 0, -1, sg->d_wb + sg->o3, no, 1, 1, sg->d_part, 0};
  LRIGW_TRY(mlp_gemm(s, g));
  hipLaunchKernelGGL(k_mlp_dtanh, dim3(nblk((long long)B * H)), dim3(256), 0, s, sg->d_part, sg->d_h2, (long long)B * H,
                     sg->d_dz2);
  // gW2 = [h1 1]^T dz2
  g = {H + 1, H, B, sg->d_h1, H, 1, H, sg->d_dz2, H, 0, 0, sg->d_part, kc};
  LRIGW_TRY(mlp_gemm(s, g));
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk((long long)(H + 1) * H)), dim3(256), 0, s, sg->d_part, S,
                     (long long)(H + 1) * H, sg->d_grad + sg->o2);
  // dz1 = (dz2 W2^T) (1 - h1^2)
  g = {B, H, H, sg->d_dz2, H, 0, -1, sg->d_wb + sg->o2, H, 1, 1, sg->d_part, 0};
  LRIGW_TRY(mlp_gemm(s, g));
  hipLaunchKernelGGL(k_mlp_dtanh, dim3(nblk((long long)B * H)), dim3(256), 0, s, sg->d_part, sg->d_h1, (long long)B * H,
                     sg->d_dz1);
  // gW1 = [x 1]^T dz1
  g = {ni + 1, H, B, xb, ni, 1, ni, sg->d_dz1, H, 0, 0, sg->d_part, kc};
  LRIGW_TRY(mlp_gemm(s, g));
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk((long long)(ni + 1) * H)), dim3(256), 0, s, sg->d_part, S,
                     (long long)(ni + 1) * H, sg->d_grad);
  return lrigw_launch_check("mlp_grad");
}

static void sur_free(lrigw_surrogate *sg) {
  void *ptrs[] = {sg->d_C, sg->d_asel, sg->d_tall, sg->d_trest, sg->d_start, sg->d_U, sg->d_Y, sg->d_G, sg->d_Linv,
                  sg->d_dinv, sg->d_T, sg->d_P, sg->d_R, sg->d_info, sg->d_theta, sg->d_m, sg->d_v, sg->d_grad, sg->d_wb,
                  sg->d_xb, sg->d_yb, sg->d_h1, sg->d_h2, sg->d_dz1, sg->d_dz2, sg->d_dy, sg->d_part, sg->d_loss_part,
                  sg->d_sig, sg->d_xdata, sg->d_ydata, sg->d_run, sg->d_nfb, sg->d_err, sg->d_nmax};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
}

static bool same_shape(const lrigw_surrogate *sg, const lrigw_ctx *c) {
  return c->d.n_aux == sg->n_aux && c->d.n_freq == sg->n_freq && c->d.x0 == sg->x0;
}

static int sur_create(lrigw_ctx *c, int rank, int n_anchor, int hidden, double d_lo, double d_hi, long long row_cap,
                      const float *init, const double *start, lrigw_surrogate **out) {
  const Dims &d = c->d;
  lrigw_surrogate *sg = new (std::nothrow) lrigw_surrogate();
  if (!sg) return LRIGW_ERR_OOM;
  sg->n_aux = d.n_aux;
  sg->n_freq = d.n_freq;
  sg->x0 = d.x0;
  sg->rank = rank;
  sg->n_anchor = n_anchor;
  sg->hidden = hidden;
  sg->d_lo = d_lo;
  sg->d_hi = d_hi;
  sg->stream = c->stream;
  for (int j = 0; j < n_anchor; ++j)
    sg->anchors.push_back((int)((2LL * j * (d.n_freq - 1) + (n_anchor - 1)) / (2LL * (n_anchor - 1))));
  sg->holdout = (sg->anchors[n_anchor / 2 - 1] + sg->anchors[n_anchor / 2]) / 2;
  for (int i = 0, l = 0; i < d.n_freq; ++i) {
    if (l < n_anchor && sg->anchors[l] == i) { ++l; continue; }
    if (i == sg->holdout) sg->t_holdout = (int)sg->targets.size();
    sg->targets.push_back(i);
  }
  sg->n_out = (int)sg->targets.size();
  const int N = d.n_aux, r = rank, H = hidden, no = sg->n_out, ni = n_anchor;
  sg->o2 = (long long)(ni + 1) * H;
  sg->o3 = sg->o2 + (long long)(H + 1) * H;
  sg->n_par = sg->o3 + (long long)(H + 1) * no;
  std::vector<double> C;
  rule_weights(c->h_omega, sg->anchors, sg->targets, d_lo, d_hi, C);
  std::vector<int> asel(sg->anchors);
  asel.push_back(sg->holdout);
  std::vector<int> trest;
  for (int t = 0; t < no; ++t)
    if (t != sg->t_holdout) trest.push_back(sg->targets[t]);
  hipStream_t s = c->stream;
  int rc = LRIGW_OK;
  auto fail = [&](int e) { rc = e; };
#define SG_TRY(expr)                                   \
  do {                                                 \
    hipError_t e__ = (expr);                           \
    if (e__ != hipSuccess) { fail(lrigw_hip_error(e__, #expr, __FILE__, __LINE__)); goto done; } \
  } while (0)
  SG_TRY(hipMalloc(&sg->d_C, C.size() * sizeof(double)));
  SG_TRY(hipMalloc(&sg->d_asel, asel.size() * sizeof(int)));
  SG_TRY(hipMalloc(&sg->d_tall, no * sizeof(int)));
  SG_TRY(hipMalloc(&sg->d_trest, std::max<size_t>(1, trest.size()) * sizeof(int)));
  SG_TRY(hipMalloc(&sg->d_start, (size_t)N * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_U, (size_t)N * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_Y, (size_t)N * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_G, (size_t)r * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_Linv, (size_t)r * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_dinv, (size_t)zdinv_stride(r) * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_T, (size_t)d.n_freq * N * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_P, (size_t)d.n_freq * r * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_R, (size_t)no * r * r * sizeof(double2)));
  SG_TRY(hipMalloc(&sg->d_info, 4 * sizeof(int)));
  SG_TRY(hipMalloc(&sg->d_theta, (size_t)sg->n_par * sizeof(float)));
  SG_TRY(hipMalloc(&sg->d_m, (size_t)sg->n_par * sizeof(float)));
  SG_TRY(hipMalloc(&sg->d_v, (size_t)sg->n_par * sizeof(float)));
  SG_TRY(hipMalloc(&sg->d_grad, (size_t)sg->n_par * sizeof(float)));
  SG_TRY(hipMalloc(&sg->d_wb, (size_t)sg->n_par * sizeof(uint16_t)));
  SG_TRY(hipMalloc(&sg->d_run, sizeof(int)));
  SG_TRY(hipMalloc(&sg->d_nfb, sizeof(int)));
  SG_TRY(hipMalloc(&sg->d_err, ERR_LOG * sizeof(double)));
  SG_TRY(hipMalloc(&sg->d_nmax, sizeof(double)));
  sg->row_cap = row_cap;
  if (row_cap > 0) {
    SG_TRY(hipMalloc(&sg->d_xdata, (size_t)row_cap * ni * sizeof(float)));
    SG_TRY(hipMalloc(&sg->d_ydata, (size_t)row_cap * no * sizeof(float)));
  }
  SG_TRY(hipMemcpyAsync(sg->d_C, C.data(), C.size() * sizeof(double), hipMemcpyHostToDevice, s));
  SG_TRY(hipMemcpyAsync(sg->d_asel, asel.data(), asel.size() * sizeof(int), hipMemcpyHostToDevice, s));
  SG_TRY(hipMemcpyAsync(sg->d_tall, sg->targets.data(), no * sizeof(int), hipMemcpyHostToDevice, s));
  if (!trest.empty()) SG_TRY(hipMemcpyAsync(sg->d_trest, trest.data(), trest.size() * sizeof(int), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_real_to_z, dim3(nblk((long long)N * r)), dim3(256), 0, s, start, (long long)N * r, sg->d_start);
  SG_TRY(hipMemcpyAsync(sg->d_theta, init, (size_t)sg->n_par * sizeof(float), hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(sg->n_par)), dim3(256), 0, s, sg->d_theta, sg->n_par, sg->d_wb);
  if ((rc = zero_fill(s, sg->d_m, (size_t)sg->n_par * sizeof(float))) < 0) goto done;
  if ((rc = zero_fill(s, sg->d_v, (size_t)sg->n_par * sizeof(float))) < 0) goto done;
  if ((rc = zero_fill(s, sg->d_nfb, sizeof(int))) < 0) goto done;
  if ((rc = zero_fill(s, sg->d_err, ERR_LOG * sizeof(double))) < 0) goto done;
  if ((rc = lrigw_launch_check("surrogate_create")) < 0) goto done;
  SG_TRY(hipStreamSynchronize(s));   // the host tables above are released on return
#undef SG_TRY
done:
  if (rc < 0) {
    sur_free(sg);
    delete sg;
    return rc;
  }
  *out = sg;
  return LRIGW_OK;
}

// ---------------------------------------------------------------- C interface
extern "C" {

int lrigw_surrogate_create(lrigw_ctx *c, int rank, int n_anchor, int hidden, double d_lo, double d_hi,
                           long long row_capacity, const float *init_params, const double *start,
                           lrigw_surrogate **out) {
  (void)hipGetLastError();
  if (!c || !out || !init_params || !start) return LRIGW_ERR_ARG;
  *out = nullptr;
  const Dims &d = c->d;
  if (n_anchor < 4 || n_anchor > 16 || d.n_freq < n_anchor + 2) return LRIGW_ERR_ARG;
  if (rank < 1 || rank > d.n_aux || rank > 256) return LRIGW_ERR_ARG;
  if (hidden < 1 || hidden > 4096 || row_capacity < 0) return LRIGW_ERR_ARG;
  if (!(d_lo > 0.0) || !(d_hi > d_lo) || !std::isfinite(d_hi)) return LRIGW_ERR_ARG;
  return sur_create(c, rank, n_anchor, hidden, d_lo, d_hi, row_capacity, init_params, start, out);
}

int lrigw_surrogate_destroy(lrigw_surrogate *sg) {
  if (!sg) return LRIGW_ERR_ARG;
  hipStreamSynchronize(sg->stream);
  sur_free(sg);
  delete sg;
  return LRIGW_OK;
}

int lrigw_surrogate_info(const lrigw_surrogate *sg, int *ints, long long *n_params) {
  if (!sg) return LRIGW_ERR_ARG;
  if (ints) {
    ints[0] = sg->n_anchor;
    ints[1] = sg->n_out;
    ints[2] = sg->holdout;
    ints[3] = sg->t_holdout;
    ints[4] = sg->rank;
    ints[5] = sg->hidden;
  }
  if (n_params) *n_params = sg->n_par;
  return LRIGW_OK;
}

int lrigw_surrogate_rule(const lrigw_surrogate *sg, double *C) {
  if (!sg || !C) return LRIGW_ERR_ARG;
  LRIGW_HIP_TRY(hipMemcpyAsync(C, sg->d_C, (size_t)sg->n_anchor * sg->n_out * sizeof(double), hipMemcpyDeviceToDevice,
                               sg->stream));
  return LRIGW_OK;
}

int lrigw_surrogate_params(lrigw_surrogate *sg, float *get, const float *set) {
  (void)hipGetLastError();
  if (!sg || (!get && !set)) return LRIGW_ERR_ARG;
  hipStream_t s = sg->stream;
  if (set) {
    LRIGW_HIP_TRY(hipMemcpyAsync(sg->d_theta, set, (size_t)sg->n_par * sizeof(float), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(sg->n_par)), dim3(256), 0, s, sg->d_theta, sg->n_par, sg->d_wb);
    LRIGW_TRY(zero_fill(s, sg->d_m, (size_t)sg->n_par * sizeof(float)));
    LRIGW_TRY(zero_fill(s, sg->d_v, (size_t)sg->n_par * sizeof(float)));
    sg->adam_t = 0;
  }
  if (get) LRIGW_HIP_TRY(hipMemcpyAsync(get, sg->d_theta, (size_t)sg->n_par * sizeof(float), hipMemcpyDeviceToDevice, s));
  return lrigw_launch_check("surrogate_params");
}

int lrigw_surrogate_basis(lrigw_surrogate *sg, lrigw_ctx *c, const void *chi_a0, void *U_out) {
  (void)hipGetLastError();
  if (!sg || !c || !chi_a0 || !U_out || !same_shape(sg, c)) return LRIGW_ERR_ARG;
  hipStream_t s = c->stream;
  const long long nn = (long long)sg->n_aux * sg->n_aux;
  // widen into the screening workspace
  if (c->precision == LRIGW_FP64)
    LRIGW_HIP_TRY(hipMemcpyAsync(c->d_s3, chi_a0, nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
  else
    hipLaunchKernelGGL(k_widen_sel<float>, dim3(nblk(nn), 1), dim3(256), 0, s, (const float2 *)chi_a0, c->d_wall, nn,
                       c->d_s3);
  LRIGW_TRY(sur_basis(sg, s, c->d_s3));
  LRIGW_HIP_TRY(hipMemcpyAsync(U_out, sg->d_U, (size_t)sg->n_aux * sg->rank * sizeof(double2), hipMemcpyDeviceToDevice, s));
  return lrigw_launch_check("surrogate_basis");
}

int lrigw_surrogate_add(lrigw_surrogate *sg, lrigw_ctx *c, const void *chi) {
  (void)hipGetLastError();
  if (!sg || !c || !chi || !same_shape(sg, c)) return LRIGW_ERR_ARG;
  const long long rr = (long long)sg->rank * sg->rank;
  if (sg->n_rows + rr > sg->row_cap) return LRIGW_ERR_ARG;
  hipStream_t s = c->stream;
  const long long nn = (long long)sg->n_aux * sg->n_aux;
  const int nw = sg->n_freq;
  if (c->precision == LRIGW_FP64)
    LRIGW_HIP_TRY(hipMemcpyAsync(c->d_s3, chi, nw * nn * sizeof(double2), hipMemcpyDeviceToDevice, s));
  else
    hipLaunchKernelGGL(k_widen_sel<float>, dim3(nblk(nn), nw), dim3(256), 0, s, (const float2 *)chi, c->d_wall, nn,
                       c->d_s3);
  LRIGW_TRY(sur_basis(sg, s, c->d_s3 + (long long)sg->anchors[0] * nn));
  LRIGW_TRY(sur_project(sg, s, c->d_s3, nw));
  hipLaunchKernelGGL(k_series_norm_max, dim3(1), dim3(1024), 0, s, sg->d_P, sg->rank, sg->d_asel, sg->n_anchor, sg->d_nmax);
  hipLaunchKernelGGL(k_series_rows, dim3(nblk(rr)), dim3(256), 0, s, sg->d_P, sg->rank, sg->d_asel, sg->n_anchor,
                     sg->d_tall, sg->n_out, sg->d_C, sg->d_nmax, sg->d_xdata + sg->n_rows * sg->n_anchor,
                     sg->d_ydata + sg->n_rows * sg->n_out);
  LRIGW_TRY(lrigw_launch_check("surrogate_add"));
  int info[2];
  LRIGW_HIP_TRY(hipMemcpyAsync(info, sg->d_info, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  LRIGW_HIP_TRY(hipStreamSynchronize(s));
  if (info[0] != INT_MAX || info[1] != INT_MAX) return LRIGW_ERR_NOT_HPD;
  sg->n_rows += rr;
  return LRIGW_OK;
}

int lrigw_surrogate_rows(lrigw_surrogate *sg, long long *n_rows, float *x, float *y, long long first, long long count) {
  if (!sg) return LRIGW_ERR_ARG;
  if (n_rows) *n_rows = sg->n_rows;
  if (x || y) {
    if (first < 0 || count < 0 || first + count > sg->n_rows) return LRIGW_ERR_ARG;
    if (x) LRIGW_HIP_TRY(hipMemcpyAsync(x, sg->d_xdata + first * sg->n_anchor, (size_t)count * sg->n_anchor * sizeof(float),
                                        hipMemcpyDeviceToDevice, sg->stream));
    if (y) LRIGW_HIP_TRY(hipMemcpyAsync(y, sg->d_ydata + first * sg->n_out, (size_t)count * sg->n_out * sizeof(float),
                                        hipMemcpyDeviceToDevice, sg->stream));
  }
  return LRIGW_OK;
}

int lrigw_surrogate_forward(lrigw_surrogate *sg, const float *x, int n_rows, float *y) {
  (void)hipGetLastError();
  if (!sg || !x || !y || n_rows < 1) return LRIGW_ERR_ARG;
  LRIGW_TRY(ensure_batch(sg, n_rows));
  LRIGW_TRY(mlp_forward(sg, sg->stream, x, n_rows));
  LRIGW_HIP_TRY(hipMemcpyAsync(y, sg->d_part, (size_t)n_rows * sg->n_out * sizeof(float), hipMemcpyDeviceToDevice,
                               sg->stream));
  return LRIGW_OK;
}

int lrigw_surrogate_grad(lrigw_surrogate *sg, const float *x, const float *y, int n_rows, float *loss, float *grad) {
  (void)hipGetLastError();
  if (!sg || !x || !y || !loss || !grad || n_rows < 1) return LRIGW_ERR_ARG;
  LRIGW_TRY(ensure_batch(sg, n_rows));
  LRIGW_TRY(mlp_grad(sg, sg->stream, x, y, n_rows, loss));
  LRIGW_HIP_TRY(hipMemcpyAsync(grad, sg->d_grad, (size_t)sg->n_par * sizeof(float), hipMemcpyDeviceToDevice, sg->stream));
  return LRIGW_OK;
}

int lrigw_surrogate_train(lrigw_surrogate *sg, int steps, int batch, double lr, const int *order, long long order_len,
                          float *loss_hist) {
  (void)hipGetLastError();
  if (!sg || !order || steps < 1 || batch < 1 || !(lr > 0.0)) return LRIGW_ERR_ARG;
  if (sg->n_rows < 1 || (long long)steps * batch > order_len) return LRIGW_ERR_ARG;
  LRIGW_TRY(ensure_batch(sg, batch));
  hipStream_t s = sg->stream;
  const double b1 = 0.9, b2 = 0.999;
  const int w = sg->n_anchor + sg->n_out;
  for (int st = 0; st < steps; ++st) {
    hipLaunchKernelGGL(k_gather_rows, dim3(nblk((long long)batch * w)), dim3(256), 0, s, sg->d_xdata, sg->d_ydata, order,
                       (long long)st * batch, batch, sg->n_anchor, sg->n_out, sg->n_rows, sg->d_xb, sg->d_yb);
    float *lo = loss_hist ? loss_hist + st : sg->d_loss_part + 0;
    LRIGW_TRY(mlp_grad(sg, s, sg->d_xb, sg->d_yb, batch, lo));
    const long long t = ++sg->adam_t;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)t)));
    hipLaunchKernelGGL(k_adam, dim3(nblk(sg->n_par)), dim3(256), 0, s, sg->d_theta, sg->d_m, sg->d_v, sg->d_grad, sg->n_par,
                       (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2, sg->d_wb);
  }
  return lrigw_launch_check("surrogate_train");
}

int lrigw_surrogate_stats(lrigw_surrogate *sg, long long *n_calls, int *n_fallback, double *errors, int max_errors) {
  if (!sg) return LRIGW_ERR_ARG;
  LRIGW_HIP_TRY(hipStreamSynchronize(sg->stream));
  if (n_calls) *n_calls = sg->n_calls;
  if (n_fallback) LRIGW_HIP_TRY(hipMemcpy(n_fallback, sg->d_nfb, sizeof(int), hipMemcpyDeviceToHost));
  if (errors && max_errors > 0) {
    long long n = std::min<long long>(std::min<long long>(sg->n_calls, ERR_LOG), max_errors);
    if (n > 0) LRIGW_HIP_TRY(hipMemcpy(errors, sg->d_err, (size_t)n * sizeof(double), hipMemcpyDeviceToHost));
  }
  return LRIGW_OK;
}

int lrigw_surrogate_reset_stats(lrigw_surrogate *sg) {
  if (!sg) return LRIGW_ERR_ARG;
  sg->n_calls = 0;
  LRIGW_TRY(zero_fill(sg->stream, sg->d_nfb, sizeof(int)));
  return LRIGW_OK;
}

}  // extern "C"

// allocations the per-q path needs, made before a graph capture
int surrogate_prepare(lrigw_surrogate *sg) { return ensure_batch(sg, sg->rank * sg->rank); }

// chi at every frequency of q: exact at the anchors and the held-out index,
// predicted elsewhere unless the held-out check fails (then exact).
int run_chi0_surrogate(lrigw_ctx *c, lrigw_surrogate *sg, int iq, const void *M, const double *eig, int apply_gamma,
                       double threshold, void *chi_out) {
  if (!same_shape(sg, c)) return LRIGW_ERR_ARG;
  if (c->gap_trusted == 0) LRIGW_TRY(chi0_check_gap(c, eig));
  GapScope gap_scope(c);
  hipStream_t s = c->stream;
  const int N = sg->n_aux, r = sg->rank, na = sg->n_anchor, no = sg->n_out;
  const long long nn = (long long)N * N, rr = (long long)r * r;
  hipEvent_t ev;
  stage_begin(c, "surrogate", &ev);
  LRIGW_TRY(run_chi0_sel(c, iq, M, eig, apply_gamma, chi_out, sg->d_asel, na + 1, nullptr));
  // FP64 copies of the anchors and the held-out response
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_widen_sel<double>, dim3(nblk(nn), na + 1), dim3(256), 0, s, (const double2 *)chi_out, sg->d_asel,
                       nn, c->d_s3);
  else
    hipLaunchKernelGGL(k_widen_sel<float>, dim3(nblk(nn), na + 1), dim3(256), 0, s, (const float2 *)chi_out, sg->d_asel,
                       nn, c->d_s3);
  LRIGW_TRY(sur_basis(sg, s, c->d_s3));
  LRIGW_TRY(sur_project(sg, s, c->d_s3, na));
  LRIGW_TRY(ensure_batch(sg, (int)rr));
  hipLaunchKernelGGL(k_series_norm_max, dim3(1), dim3(1024), 0, s, sg->d_P, r, nullptr, na, sg->d_nmax);
  hipLaunchKernelGGL(k_series_features, dim3(nblk(rr)), dim3(256), 0, s, sg->d_P, r, na, sg->d_nmax, sg->d_xb, sg->d_sig);
  LRIGW_TRY(mlp_forward(sg, s, sg->d_xb, (int)rr));
  hipLaunchKernelGGL(k_series_residual, dim3(nblk(rr * no)), dim3(256), 0, s, sg->d_part, sg->d_sig, r, no, sg->d_R);
  // T1[t] = U R_t (into d_T), T2[t] = T1[t] U^H (into the screening workspace s0)
  const double2 one = mkc(1.0, 0.0);
  LRIGW_TRY(zgemm(s, zg(N, r, r, OP_N, sg->d_U, r, 0, OP_N, sg->d_R, r, rr, sg->d_T, r, (long long)N * r, one, no)));
  LRIGW_TRY(zgemm(s, zg(N, N, r, OP_N, sg->d_T, r, (long long)N * r, OP_C, sg->d_U, r, 0, c->d_s0, N, nn, one, no)));
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_sur_combine<double>, dim3(nblk(nn), no), dim3(256), 0, s, c->d_s3, na, sg->d_C, no, c->d_s0,
                       sg->d_tall, sg->t_holdout, nn, (double2 *)chi_out, c->d_s1);
  else
    hipLaunchKernelGGL(k_sur_combine<float>, dim3(nblk(nn), no), dim3(256), 0, s, c->d_s3, na, sg->d_C, no, c->d_s0,
                       sg->d_tall, sg->t_holdout, nn, (float2 *)chi_out, c->d_s1);
  hipLaunchKernelGGL(k_sur_check, dim3(1), dim3(1024), 0, s, c->d_s1, c->d_s3 + (long long)na * nn, nn, threshold,
                     sg->d_run, sg->d_nfb, sg->d_err, sg->n_calls);
  sg->n_calls += 1;
  LRIGW_TRY(lrigw_launch_check("surrogate_predict"));
  if (no > 1) LRIGW_TRY(run_chi0_sel(c, iq, M, eig, apply_gamma, chi_out, sg->d_trest, no - 1, sg->d_run));
  stage_end(c, "surrogate", ev);
  return LRIGW_OK;
}
