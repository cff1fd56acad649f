// Dense FP64 complex building blocks: batched GEMM, blocked Cholesky and
// triangular solves (used by the screening step and the LRI half-transform).
#include <algorithm>
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

#define GT 64      // output tile
#define GK 8       // K step

__device__ inline double2 ldop(const double2 *__restrict__ A, long long ld, int op, long long r, long long cidx) {
  // element (r, cidx) of op(A)
  if (op == OP_N) return A[r * ld + cidx];
  double2 v = A[cidx * ld + r];
  if (op == OP_C) v.y = -v.y;
  return v;
}

// C = alpha op(A) op(B) + beta C, 64x64 tile per workgroup, 4x4 outputs per thread.
__global__ __launch_bounds__(256) void k_zgemm(ZGemm g) {
  __shared__ double2 As[GK][GT + 1];
  __shared__ double2 Bs[GK][GT + 1];
  const int tm = blockIdx.x, tn = blockIdx.y, b = blockIdx.z;
  const int m0 = tm * GT, n0 = tn * GT;
  if (g.lower_only && n0 > m0 + GT - 1) return;
  const double2 *A = g.A + (long long)b * g.sa;
  const double2 *B = g.B + (long long)b * g.sb;
  double2 *C = g.C + (long long)b * g.sc;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double cr[4][4], ci[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) cr[i][j] = ci[i][j] = 0.0;
  for (int k0 = 0; k0 < g.k; k0 += GK) {
#pragma unroll
    for (int t = 0; t < (GK * GT) / 256; ++t) {
      int e = tid + 256 * t;
      // A tile: rows m0..m0+63, cols k0..k0+7 ; choose the mapping that walks memory contiguously
      int kk, mm;
      if (g.opa == OP_N) { mm = e / GK; kk = e % GK; } else { kk = e / GT; mm = e % GT; }
      double2 v = mkc(0.0, 0.0);
      if (m0 + mm < g.m && k0 + kk < g.k) v = ldop(A, g.lda, g.opa, m0 + mm, k0 + kk);
      As[kk][mm] = v;
      int nn;
      if (g.opb == OP_N) { kk = e / GT; nn = e % GT; } else { nn = e / GK; kk = e % GK; }
      double2 u = mkc(0.0, 0.0);
      if (n0 + nn < g.n && k0 + kk < g.k) u = ldop(B, g.ldb, g.opb, k0 + kk, n0 + nn);
      Bs[kk][nn] = u;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double2 a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          cr[i][j] += a[i].x * bb[j].x - a[i].y * bb[j].y;
          ci[i][j] += a[i].x * bb[j].y + a[i].y * bb[j].x;
        }
    }
    __syncthreads();
  }
  const bool beta0 = (g.beta.x == 0.0 && g.beta.y == 0.0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int r = m0 + ty + 16 * i;
    if (r >= g.m) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int cc = n0 + tx + 16 * j;
      if (cc >= g.n) continue;
      if (g.lower_only && cc > r) continue;
      double2 v = mkc(g.alpha.x * cr[i][j] - g.alpha.y * ci[i][j], g.alpha.x * ci[i][j] + g.alpha.y * cr[i][j]);
      long long o = (long long)r * g.ldc + cc;
      if (!beta0) {
        double2 old = C[o];
        v.x += g.beta.x * old.x - g.beta.y * old.y;
        v.y += g.beta.x * old.y + g.beta.y * old.x;
      }
      C[o] = v;
    }
  }
}

int zgemm(hipStream_t s, const ZGemm &g) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return LRIGW_OK;
  if (g.k <= 0) {
    // C = beta C: not needed by the callers
    return LRIGW_ERR_ARG;
  }
  dim3 grid((g.m + GT - 1) / GT, (g.n + GT - 1) / GT, g.batch);
  hipLaunchKernelGGL(k_zgemm, grid, dim3(256), 0, s, g);
  return lrigw_launch_check("zgemm");
}

// ---------------------------------------------------------------- Cholesky
#define NB 32

// Factor the jb x jb diagonal block at (j0, j0) of every matrix in LDS.
__global__ __launch_bounds__(256) void k_potrf_diag(double2 *A, long long lda, long long stride, int j0, int jb, int *info) {
  __shared__ double2 L[NB][NB + 1];
  __shared__ int bad;
  double2 *M = A + (long long)blockIdx.x * stride;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e / jb, cc = e % jb;
    L[r][cc] = M[(long long)(j0 + r) * lda + j0 + cc];
  }
  __syncthreads();
  for (int cc = 0; cc < jb; ++cc) {
    if (tid == 0) {
      double p = L[cc][cc].x;
      if (!(p > 0.0) || !isfinite(p)) {
        bad = 1;
        p = 1.0;
      }
      L[cc][cc] = mkc(sqrt(p), 0.0);
    }
    __syncthreads();
    const double dinv = 1.0 / L[cc][cc].x;
    for (int r = cc + 1 + tid; r < jb; r += blockDim.x) {
      L[r][cc].x *= dinv;
      L[r][cc].y *= dinv;
    }
    __syncthreads();
    // trailing update of the lower part: L[r][s] -= L[r][cc] conj(L[s][cc]), cc < s <= r
    const int rem = jb - cc - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      int r = cc + 1 + e / rem, s2 = cc + 1 + e % rem;
      if (s2 <= r) {
        double2 a = L[r][cc], b = L[s2][cc];
        L[r][s2].x -= a.x * b.x + a.y * b.y;
        L[r][s2].y -= a.y * b.x - a.x * b.y;
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    int r = e / jb, cc = e % jb;
    M[(long long)(j0 + r) * lda + j0 + cc] = (cc <= r) ? L[r][cc] : mkc(0.0, 0.0);
  }
  if (tid == 0 && bad) atomicMin(info + 0, blockIdx.x);
}

// Panel: A[r][j0..j0+jb) <- A[r][..] L_jj^{-H} for rows r >= j0+jb (one thread per row).
__global__ __launch_bounds__(256) void k_trsm_panel(double2 *A, long long lda, long long stride, int n, int j0, int jb) {
  __shared__ double2 L[NB][NB + 1];
  double2 *M = A + (long long)blockIdx.y * stride;
  for (int e = threadIdx.x; e < jb * jb; e += blockDim.x) L[e / jb][e % jb] = M[(long long)(j0 + e / jb) * lda + j0 + e % jb];
  __syncthreads();
  int r = j0 + jb + blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double2 x[NB];
  double2 *row = M + (long long)r * lda + j0;
  for (int cc = 0; cc < jb; ++cc) {
    // x L^H = a  ->  x_c = (a_c - sum_{t<c} x_t conj(L[c][t])) / L[c][c]
    double2 v = row[cc];
    for (int t = 0; t < cc; ++t) {
      double2 l = L[cc][t];
      v.x -= x[t].x * l.x + x[t].y * l.y;
      v.y -= x[t].y * l.x - x[t].x * l.y;
    }
    double dinv = 1.0 / L[cc][cc].x;
    x[cc] = mkc(v.x * dinv, v.y * dinv);
  }
  for (int cc = 0; cc < jb; ++cc) row[cc] = x[cc];
}

__global__ void k_zero_upper(double2 *A, long long lda, long long stride, int n) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  int r = (int)(idx / n), cc = (int)(idx % n);
  if (cc > r) A[(long long)blockIdx.y * stride + (long long)r * lda + cc] = mkc(0.0, 0.0);
}

__global__ void k_info_init(int *info, int v) { info[threadIdx.x] = v; }

// A = L L^H in place (lower; the strict upper part is zeroed).  d_info[0] = first
// failing batch index, or INT_MAX.
int zpotrf_batched(hipStream_t s, double2 *A, int n, long long lda, long long stride, int batch, int *d_info) {
  hipLaunchKernelGGL(k_info_init, dim3(1), dim3(1), 0, s, d_info, 0x7fffffff);
  for (int j0 = 0; j0 < n; j0 += NB) {
    int jb = std::min(NB, n - j0);
    hipLaunchKernelGGL(k_potrf_diag, dim3(batch), dim3(256), 0, s, A, lda, stride, j0, jb, d_info);
    int rest = n - j0 - jb;
    if (rest > 0) {
      hipLaunchKernelGGL(k_trsm_panel, dim3((rest + 255) / 256, batch), dim3(256), 0, s, A, lda, stride, n, j0, jb);
      ZGemm g;
      g.m = rest;
      g.n = rest;
      g.k = jb;
      g.opa = OP_N;
      g.A = A + (long long)(j0 + jb) * lda + j0;
      g.lda = lda;
      g.sa = stride;
      g.opb = OP_C;
      g.B = A + (long long)(j0 + jb) * lda + j0;
      g.ldb = lda;
      g.sb = stride;
      g.C = A + (long long)(j0 + jb) * lda + j0 + jb;
      g.ldc = lda;
      g.sc = stride;
      g.alpha = mkc(-1.0, 0.0);
      g.beta = mkc(1.0, 0.0);
      g.batch = batch;
      g.lower_only = 1;
      LRIGW_TRY(zgemm(s, g));
    }
  }
  dim3 zg((unsigned)(((long long)n * n + 255) / 256), batch);
  hipLaunchKernelGGL(k_zero_upper, zg, dim3(256), 0, s, A, lda, stride, n);
  return lrigw_launch_check("zpotrf");
}

// ---------------------------------------------------------------- triangular solves, full right-hand sides
// rows j0..j0+jb of Y <- L_jj^{-1} rows (forward), one thread per column
__global__ __launch_bounds__(256) void k_trsm_lower_diag(const double2 *L, long long ldl, long long sl, double2 *Y, long long ldy,
                                                         long long sy, int j0, int jb, int ncols) {
  __shared__ double2 Ld[NB][NB + 1];
  const double2 *Lb = L + (long long)blockIdx.y * sl;
  for (int e = threadIdx.x; e < jb * jb; e += blockDim.x) Ld[e / jb][e % jb] = Lb[(long long)(j0 + e / jb) * ldl + j0 + e % jb];
  __syncthreads();
  int cc = blockIdx.x * blockDim.x + threadIdx.x;
  if (cc >= ncols) return;
  double2 *Yb = Y + (long long)blockIdx.y * sy;
  double2 y[NB];
  for (int r = 0; r < jb; ++r) {
    double2 v = Yb[(long long)(j0 + r) * ldy + cc];
    for (int t = 0; t < r; ++t) {
      double2 l = Ld[r][t];
      v.x -= l.x * y[t].x - l.y * y[t].y;
      v.y -= l.x * y[t].y + l.y * y[t].x;
    }
    double dinv = 1.0 / Ld[r][r].x;
    y[r] = mkc(v.x * dinv, v.y * dinv);
  }
  for (int r = 0; r < jb; ++r) Yb[(long long)(j0 + r) * ldy + cc] = y[r];
}

// rows j0..j0+jb of Y <- L_jj^{-H} rows (backward), one thread per column
__global__ __launch_bounds__(256) void k_trsm_upperc_diag(const double2 *L, long long ldl, long long sl, double2 *Y, long long ldy,
                                                          long long sy, int j0, int jb, int ncols) {
  __shared__ double2 Ld[NB][NB + 1];
  const double2 *Lb = L + (long long)blockIdx.y * sl;
  for (int e = threadIdx.x; e < jb * jb; e += blockDim.x) Ld[e / jb][e % jb] = Lb[(long long)(j0 + e / jb) * ldl + j0 + e % jb];
  __syncthreads();
  int cc = blockIdx.x * blockDim.x + threadIdx.x;
  if (cc >= ncols) return;
  double2 *Yb = Y + (long long)blockIdx.y * sy;
  double2 y[NB];
  for (int r = jb - 1; r >= 0; --r) {
    double2 v = Yb[(long long)(j0 + r) * ldy + cc];
    for (int t = r + 1; t < jb; ++t) {
      double2 l = Ld[t][r];  // (L^H)[r][t] = conj(L[t][r])
      v.x -= l.x * y[t].x + l.y * y[t].y;
      v.y -= l.x * y[t].y - l.y * y[t].x;
    }
    double dinv = 1.0 / Ld[r][r].x;
    y[r] = mkc(v.x * dinv, v.y * dinv);
  }
  for (int r = 0; r < jb; ++r) Yb[(long long)(j0 + r) * ldy + cc] = y[r];
}

// Y <- L^{-1} Y  (L lower, n x n; Y n x ncols)
int ztrsm_left_lower(hipStream_t s, const double2 *L, long long ldl, long long sl, double2 *Y, long long ldy, long long sy,
                     int n, int ncols, int batch) {
  for (int j0 = 0; j0 < n; j0 += NB) {
    int jb = std::min(NB, n - j0);
    if (j0 > 0) {
      ZGemm g;
      g.m = jb;
      g.n = ncols;
      g.k = j0;
      g.opa = OP_N;
      g.A = L + (long long)j0 * ldl;
      g.lda = ldl;
      g.sa = sl;
      g.opb = OP_N;
      g.B = Y;
      g.ldb = ldy;
      g.sb = sy;
      g.C = Y + (long long)j0 * ldy;
      g.ldc = ldy;
      g.sc = sy;
      g.alpha = mkc(-1.0, 0.0);
      g.beta = mkc(1.0, 0.0);
      g.batch = batch;
      g.lower_only = 0;
      LRIGW_TRY(zgemm(s, g));
    }
    hipLaunchKernelGGL(k_trsm_lower_diag, dim3((ncols + 255) / 256, batch), dim3(256), 0, s, L, ldl, sl, Y, ldy, sy, j0, jb,
                       ncols);
  }
  return lrigw_launch_check("ztrsm_lower");
}

// Y <- L^{-H} Y
int ztrsm_left_upper_conj(hipStream_t s, const double2 *L, long long ldl, long long sl, double2 *Y, long long ldy, long long sy,
                          int n, int ncols, int batch) {
  int nblk = (n + NB - 1) / NB;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    int j0 = bi * NB;
    int jb = std::min(NB, n - j0);
    int rest = n - j0 - jb;
    if (rest > 0) {
      // Y[j0..] -= (L[j0+jb.., j0..j0+jb))^H Y[j0+jb..]
      ZGemm g;
      g.m = jb;
      g.n = ncols;
      g.k = rest;
      g.opa = OP_C;
      g.A = L + (long long)(j0 + jb) * ldl + j0;
      g.lda = ldl;
      g.sa = sl;
      g.opb = OP_N;
      g.B = Y + (long long)(j0 + jb) * ldy;
      g.ldb = ldy;
      g.sb = sy;
      g.C = Y + (long long)j0 * ldy;
      g.ldc = ldy;
      g.sc = sy;
      g.alpha = mkc(-1.0, 0.0);
      g.beta = mkc(1.0, 0.0);
      g.batch = batch;
      g.lower_only = 0;
      LRIGW_TRY(zgemm(s, g));
    }
    hipLaunchKernelGGL(k_trsm_upperc_diag, dim3((ncols + 255) / 256, batch), dim3(256), 0, s, L, ldl, sl, Y, ldy, sy, j0, jb,
                       ncols);
  }
  return lrigw_launch_check("ztrsm_upperc");
}
