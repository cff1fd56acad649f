// Dense FP64 complex building blocks: batched GEMM on FP64 MFMA, blocked
// Cholesky and triangular solves (screening step, LRI half-transform).
#include <algorithm>
#include <climits>
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

#define GT 64      // output tile
#define GK 16      // K rows staged per step
#define GP (GT + 1)

// C = alpha op(A) op(B) + beta C; 64x64 tile per workgroup, four waves of
// 32x32, complex products as four real FP64 MFMA 16x16x4 products.  The ops
// are template parameters, so the staging loads have no branches: elements
// outside the matrices come from index 0 and are replaced by zero after the
// load, and the next K step is fetched into registers while the current one
// is multiplied.  A workgroup reads all of op(A)'s rows and op(B)'s columns of
// its tile before it writes the tile, so C may alias A when n <= 64 or B when
// m <= 64.
template <int OPA, int OPB>
__global__ __launch_bounds__(256) void k_zgemm(ZGemm g) {
  typedef Mfma<double> MF;
  __shared__ double2 As[GK][GP];   // As[k][m] = op(A)(m0+m, k0+k)
  __shared__ double2 Bs[GK][GP];   // Bs[k][n] = op(B)(k0+k, n0+n)
  const int tm = blockIdx.x, tn = blockIdx.y, b = blockIdx.z;
  const int m0 = tm * GT, n0 = tn * GT;
  if (g.lower_only && n0 > m0 + GT - 1) return;
  const double2 *A = g.A + (long long)(b % g.bdiv) * g.sa + (long long)(b / g.bdiv) * g.sa2;
  const double2 *B = g.B + (long long)(b % g.bdiv) * g.sb + (long long)(b / g.bdiv) * g.sb2;
  double2 *C = g.C + (long long)b * g.sc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, col = lane & 15;
  const double2 zero = mkc(0.0, 0.0);
  // 16x16 blocks of this wave that hold any output (a tile of the last tile
  // row or column is mostly padding; the others' products are skipped)
  const bool rin[2] = {m0 + 32 * wr < g.m, m0 + 32 * wr + 16 < g.m};
  const bool cin[2] = {n0 + 32 * wc < g.n, n0 + 32 * wc + 16 < g.n};
  d4v cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) cr[i][j] = ci[i][j] = MF::zero();
  // staging map: along the contiguous index of each operand
  double2 ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int t = 0; t < (GK * GT) / 256; ++t) {
      const int e = tid + 256 * t;
      {
        const int mm = OPA == OP_N ? e / GK : e % GT, kk = OPA == OP_N ? e % GK : e / GT;
        const bool ok = m0 + mm < g.m && k0 + kk < g.k;
        const long long idx = OPA == OP_N ? (long long)(m0 + mm) * g.lda + k0 + kk : (long long)(k0 + kk) * g.lda + m0 + mm;
        double2 v = ld_or(A, idx, ok, zero);
        if (OPA == OP_C) v.y = -v.y;
        ra[t] = v;
      }
      {
        const int nn = OPB == OP_N ? e % GT : e / GK, kk = OPB == OP_N ? e / GT : e % GK;
        const bool ok = n0 + nn < g.n && k0 + kk < g.k;
        const long long idx = OPB == OP_N ? (long long)(k0 + kk) * g.ldb + n0 + nn : (long long)(n0 + nn) * g.ldb + k0 + kk;
        double2 u = ld_or(B, idx, ok, zero);
        if (OPB == OP_C) u.y = -u.y;
        rb[t] = u;
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int t = 0; t < (GK * GT) / 256; ++t) {
      const int e = tid + 256 * t;
      const int mm = OPA == OP_N ? e / GK : e % GT, ka = OPA == OP_N ? e % GK : e / GT;
      As[ka][mm] = ra[t];
      const int nn = OPB == OP_N ? e % GT : e / GK, kb = OPB == OP_N ? e / GT : e % GK;
      Bs[kb][nn] = rb[t];
    }
  };
  // K range this tile needs when an operand is triangular (the skipped
  // products are with stored zeros; both ends are multiples of GT)
  int k_lo = 0, k_hi = g.k;
  if (g.tri_b == TRI_LOWER) k_lo = max(k_lo, n0);        // op(B)[k][c] = 0 for k < c
  if (g.tri_b == TRI_UPPER) k_hi = min(k_hi, n0 + GT);   // op(B)[k][c] = 0 for k > c
  if (g.tri_a == TRI_UPPER) k_lo = max(k_lo, m0);        // op(A)[r][k] = 0 for k < r
  if (g.tri_a == TRI_LOWER) k_hi = min(k_hi, m0 + GT);   // op(A)[r][k] = 0 for k > r
  fetch(k_lo);
  for (int k0 = k_lo; k0 < k_hi; k0 += GK) {
    __syncthreads();
    stash();
    __syncthreads();
    fetch(k0 + GK);   // past the end: all zero, harmless
#pragma unroll
    for (int ks = 0; ks < GK / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double2 a[2], bb[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        a[s] = As[kk][32 * wr + 16 * s + col];
        bb[s] = Bs[kk][32 * wc + 16 * s + col];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (!rin[i] || !cin[j]) continue;
          cr[i][j] = MF::mac(a[i].x, bb[j].x, cr[i][j]);
          ci[i][j] = MF::mac(a[i].x, bb[j].y, ci[i][j]);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          if (!rin[i] || !cin[j]) continue;
          cr[i][j] = MF::mac(-a[i].y, bb[j].y, cr[i][j]);
          ci[i][j] = MF::mac(a[i].y, bb[j].x, ci[i][j]);
        }
    }
  }
  __syncthreads();   // every read of an aliased operand is done before any write
  const bool beta0 = (g.beta.x == 0.0 && g.beta.y == 0.0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = m0 + 32 * wr + 16 * i + MF::row(lane, q);
        const int cc = n0 + 32 * wc + 16 * j + col;
        if (r >= g.m || cc >= g.n) continue;
        if (g.lower_only && cc > r) continue;
        const double xr = cr[i][j][q], xi = ci[i][j][q];
        double2 v = mkc(g.alpha.x * xr - g.alpha.y * xi, g.alpha.x * xi + g.alpha.y * xr);
        const long long o = (long long)r * g.ldc + cc;
        if (!beta0) {
          const double2 old = C[o];
          v.x += g.beta.x * old.x - g.beta.y * old.y;
          v.y += g.beta.x * old.y + g.beta.y * old.x;
        }
        C[o] = v;
      }
}

int zgemm(hipStream_t s, const ZGemm &g) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return LRIGW_OK;
  if (g.k <= 0) return LRIGW_ERR_ARG;
  if (g.opa < OP_N || g.opa > OP_C || g.opb < OP_N || g.opb > OP_C) return LRIGW_ERR_ARG;
  dim3 grid((g.m + GT - 1) / GT, (g.n + GT - 1) / GT, g.batch);
#define ZG(OA, OB) \
  if (g.opa == OA && g.opb == OB) hipLaunchKernelGGL((k_zgemm<OA, OB>), grid, dim3(256), 0, s, g);
  ZG(OP_N, OP_N) ZG(OP_N, OP_T) ZG(OP_N, OP_C)
  ZG(OP_T, OP_N) ZG(OP_T, OP_T) ZG(OP_T, OP_C)
  ZG(OP_C, OP_N) ZG(OP_C, OP_T) ZG(OP_C, OP_C)
#undef ZG
  return lrigw_launch_check("zgemm");
}

// ---------------------------------------------------------------- Cholesky, NB = 64
#define NB 64
#define NBP (NB + 1)

// Factor the jb x jb diagonal block at (j0, j0) of every matrix in LDS, write
// back L_jj (lower, strict upper zeroed) and its inverse into
// Dinv[batch][blk][NB][NB].  info[0] = smallest failing batch index.
__global__ __launch_bounds__(256) void k_potrf_diag(double2 *A, long long lda, long long stride, int j0, int jb, double2 *Dinv,
                                                    long long dstride, int *info) {
  __shared__ double2 L[NB][NBP];
  __shared__ double2 X[NB][NBP];
  __shared__ int bad;
  double2 *M = A + (long long)blockIdx.x * stride;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    const int r = e / jb, cc = e % jb;
    L[r][cc] = M[(long long)(j0 + r) * lda + j0 + cc];
  }
  __syncthreads();
  // right-looking LDL^H on the unscaled columns (one barrier per column):
  // d_cc = L[cc][cc];  L[r][s] -= L[r][cc] conj(L[s][cc]) / d_cc  (cc < s <= r)
  __shared__ double piv[NB];
  for (int cc = 0; cc < jb; ++cc) {
    double p = L[cc][cc].x;
    if (!(p > 0.0) || !isfinite(p)) {
      if (tid == 0) bad = 1;
      p = 1.0;
    }
    if (tid == 0) piv[cc] = p;
    const double pinv = 1.0 / p;
    // 16 x 16 thread grid over the trailing lower triangle
    for (int r = cc + 1 + (tid >> 4); r < jb; r += 16) {
      const double2 a = L[r][cc];
      for (int s2 = cc + 1 + (tid & 15); s2 <= r; s2 += 16) {
        const double2 b = L[s2][cc];
        L[r][s2].x -= (a.x * b.x + a.y * b.y) * pinv;
        L[r][s2].y -= (a.y * b.x - a.x * b.y) * pinv;
      }
    }
    __syncthreads();
  }
  // Cholesky factor: column cc scaled by 1/sqrt(d_cc), diagonal sqrt(d_cc)
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    const int r = e / jb, cc = e % jb;
    if (cc < r) {
      const double sinv = 1.0 / sqrt(piv[cc]);
      L[r][cc].x *= sinv;
      L[r][cc].y *= sinv;
    } else if (cc == r) {
      L[r][r] = mkc(sqrt(piv[r]), 0.0);
    }
  }
  __syncthreads();
  // inverse of the lower-triangular block by forward substitution, column j
  // by four adjacent lanes: X[i][j] = (delta_ij - sum_{t=j}^{i-1} L[i][t] X[t][j]) / L[i][i];
  // lane part sums the t with t = part (mod 4) and writes the rows i = part
  // (mod 4), so every X entry a lane reads is one it wrote itself.
  {
    const int j = tid >> 2, part = tid & 3;
    const bool act = j < jb;
    for (int i = 0; i < jb; ++i) {
      double sr = 0.0, si = 0.0;
      if (act && i > j) {
        for (int t = j + ((part - j) & 3); t < i; t += 4) {
          const double2 l = L[i][t], x = X[t][j];
          sr += l.x * x.x - l.y * x.y;
          si += l.x * x.y + l.y * x.x;
        }
      }
      sr += __shfl_xor(sr, 1);
      si += __shfl_xor(si, 1);
      sr += __shfl_xor(sr, 2);
      si += __shfl_xor(si, 2);
      if (act && (i & 3) == part) {
        if (i < j) {
          X[i][j] = mkc(0.0, 0.0);
        } else {
          const double dinv = 1.0 / L[i][i].x;
          X[i][j] = mkc(((i == j ? 1.0 : 0.0) - sr) * dinv, -si * dinv);
        }
      }
    }
  }
  __syncthreads();
  double2 *D = Dinv + (long long)blockIdx.x * dstride + (long long)(j0 / NB) * NB * NB;
  for (int e = tid; e < jb * jb; e += blockDim.x) {
    const int r = e / jb, cc = e % jb;
    M[(long long)(j0 + r) * lda + j0 + cc] = (cc <= r) ? L[r][cc] : mkc(0.0, 0.0);
    D[r * NB + cc] = X[r][cc];
  }
  if (tid == 0 && bad) atomicMin(info + 0, blockIdx.x);
}

__global__ void k_zero_upper(double2 *A, long long lda, long long stride, int n) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)n * n) return;
  const int r = (int)(idx / n), cc = (int)(idx % n);
  if (cc > r) A[(long long)blockIdx.y * stride + (long long)r * lda + cc] = mkc(0.0, 0.0);
}

__global__ void k_info_init(int *info, int v) { info[threadIdx.x] = v; }

static ZGemm mkg(int m, int n, int k, int opa, const double2 *A, long long lda, long long sa, int opb, const double2 *B,
                 long long ldb, long long sb, double2 *Cm, long long ldc, long long sc, double2 alpha, double2 beta,
                 int batch, int lower_only) {
  ZGemm g;
  g.m = m; g.n = n; g.k = k;
  g.opa = opa; g.A = A; g.lda = lda; g.sa = sa;
  g.opb = opb; g.B = B; g.ldb = ldb; g.sb = sb;
  g.C = Cm; g.ldc = ldc; g.sc = sc;
  g.alpha = alpha; g.beta = beta;
  g.batch = batch; g.lower_only = lower_only;
  return g;
}

long long zdinv_stride(int n) { return (long long)((n + NB - 1) / NB) * NB * NB; }

// A = L L^H in place (lower; strict upper part zeroed); Dinv receives the
// inverses of the diagonal blocks (zdinv_stride(n) elements per matrix).
// d_info[0] = first failing batch index, or INT_MAX.
int zpotrf_batched(hipStream_t s, double2 *A, int n, long long lda, long long stride, int batch, double2 *Dinv, int *d_info) {
  const long long ds = zdinv_stride(n);
  const double2 one = mkc(1.0, 0.0), mone = mkc(-1.0, 0.0), zero = mkc(0.0, 0.0);
  hipLaunchKernelGGL(k_info_init, dim3(1), dim3(1), 0, s, d_info, INT_MAX);
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = std::min(NB, n - j0);
    hipLaunchKernelGGL(k_potrf_diag, dim3(batch), dim3(256), 0, s, A, lda, stride, j0, jb, Dinv, ds, d_info);
    const int rest = n - j0 - jb;
    if (rest > 0) {
      double2 *P = A + (long long)(j0 + jb) * lda + j0;
      const double2 *D = Dinv + (long long)(j0 / NB) * NB * NB;
      // panel P <- P L_jj^{-H} (in place: one column tile)
      LRIGW_TRY(zgemm(s, mkg(rest, jb, jb, OP_N, P, lda, stride, OP_C, D, NB, ds, P, lda, stride, one, zero, batch, 0)));
      // trailing update, lower part: A22 -= P P^H
      LRIGW_TRY(zgemm(s, mkg(rest, rest, jb, OP_N, P, lda, stride, OP_C, P, lda, stride, P + jb, lda, stride, mone, one,
                          batch, 1)));
    }
  }
  dim3 zg((unsigned)(((long long)n * n + 255) / 256), batch);
  hipLaunchKernelGGL(k_zero_upper, zg, dim3(256), 0, s, A, lda, stride, n);
  return lrigw_launch_check("zpotrf");
}

// Y <- L^{-1} Y  (L lower n x n with Dinv from zpotrf_batched; Y n x ncols)
int ztrsm_left_lower(hipStream_t s, const double2 *L, long long ldl, long long sl, const double2 *Dinv, double2 *Y,
                     long long ldy, long long sy, int n, int ncols, int batch) {
  const long long ds = zdinv_stride(n);
  const double2 one = mkc(1.0, 0.0), mone = mkc(-1.0, 0.0), zero = mkc(0.0, 0.0);
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = std::min(NB, n - j0);
    double2 *Yj = Y + (long long)j0 * ldy;
    if (j0 > 0)
      LRIGW_TRY(zgemm(s, mkg(jb, ncols, j0, OP_N, L + (long long)j0 * ldl, ldl, sl, OP_N, Y, ldy, sy, Yj, ldy, sy, mone,
                          one, batch, 0)));
    // Y_j <- L_jj^{-1} Y_j (in place: one row tile)
    LRIGW_TRY(zgemm(s, mkg(jb, ncols, jb, OP_N, Dinv + (long long)(j0 / NB) * NB * NB, NB, ds, OP_N, Yj, ldy, sy, Yj, ldy,
                        sy, one, zero, batch, 0)));
  }
  return LRIGW_OK;
}

// Y <- L^{-H} Y
int ztrsm_left_upper_conj(hipStream_t s, const double2 *L, long long ldl, long long sl, const double2 *Dinv, double2 *Y,
                          long long ldy, long long sy, int n, int ncols, int batch) {
  const long long ds = zdinv_stride(n);
  const double2 one = mkc(1.0, 0.0), mone = mkc(-1.0, 0.0), zero = mkc(0.0, 0.0);
  const int nblk = (n + NB - 1) / NB;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int j0 = bi * NB;
    const int jb = std::min(NB, n - j0);
    const int rest = n - j0 - jb;
    double2 *Yj = Y + (long long)j0 * ldy;
    if (rest > 0)
      LRIGW_TRY(zgemm(s, mkg(jb, ncols, rest, OP_C, L + (long long)(j0 + jb) * ldl + j0, ldl, sl, OP_N,
                          Y + (long long)(j0 + jb) * ldy, ldy, sy, Yj, ldy, sy, mone, one, batch, 0)));
    // Y_j <- L_jj^{-H} Y_j
    LRIGW_TRY(zgemm(s, mkg(jb, ncols, jb, OP_C, Dinv + (long long)(j0 / NB) * NB * NB, NB, ds, OP_N, Yj, ldy, sy, Yj, ldy,
                        sy, one, zero, batch, 0)));
  }
  return LRIGW_OK;
}
