// Correlation self-energy (Eq. GW_selfe_element with W -> W^c, w_q = 1/N_q).
//
// Pair weights X_c(w) = sum_{mu nu} x_c^mu W^c_{mu nu}(w) conj(x_c^nu) for every
// column c = (k, n, m), with W^c Hermitian:
//   X_c = sum_mu Re W_{mu mu} |x_mu|^2 + 2 Re sum_mu x_mu Z_mu,
//   Z_mu = sum_{nu < mu} W_{mu nu} conj(x_nu),
// so only the strictly lower 64x64 blocks of W^c enter the MFMA product and the
// reduction over mu finishes inside the workgroup (no atomics).  A second
// kernel contracts X with the folded frequency kernel in FP64.
#include <algorithm>
#include <vector>
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

#define SKC 16          // nu rows staged per step

// Workgroup -> (column block, frequency block).  Consecutive workgroup ids go
// to different XCDs (id mod 8).  Each XCD owns a fixed set of ceil(nfb/8)
// frequency blocks and walks all column blocks with them, so the W^c of its
// frequencies (a few MB) stays in that XCD's L2 while x streams through once
// per XCD; the frequency blocks of one column block run back to back and share
// the x tile.
__device__ inline bool xcd_map(int nfb, long long ncb, long long &cb, int &fb) {
  const long long b = blockIdx.x;
  const long long slot = b >> 3;
  const int fpx = (nfb + 7) >> 3;
  fb = (int)(b & 7) * fpx + (int)(slot % fpx);
  cb = slot / fpx;
  return cb < ncb && fb < nfb;
}
static inline unsigned xcd_grid(int nfb, long long ncb) { return (unsigned)(8LL * ((nfb + 7) / 8) * ncb); }
#define SLP (TILE + 1)  // padded LDS row (complex elements)

// One workgroup = 64 columns c (x rows) and every row mu of W^c.  Rows are
// taken in groups of 64 aligned to the END of the range (the ragged group is
// the first and costs the least); wave w owns rows 16w..16w+15 of a group and
// all 64 columns (4 MFMA column tiles).  The contraction index nu runs in
// chunks of 16 from 0 to the diagonal (strictly lower part only); LDS is double
// buffered and the next chunk is fetched into registers while the current one
// is multiplied.  The reduction over mu is accumulated in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_sigma_mfma(const typename c2t<T>::type *__restrict__ x, const typename c2t<T>::type *__restrict__ Wall,
                                                    long long Ccols, int N, int n_freq, double *__restrict__ Xall) {
  typedef typename c2t<T>::type C;
  typedef Mfma<T> MF;
  typedef typename MF::acc ACC;
  __shared__ C Ws[2][SKC][SLP];   // Ws[b][nu][mu] = W[mu][nu] for the current group
  __shared__ C Us[2][SKC][SLP];   // Us[b][nu][c]  = conj(x[c][nu])
  __shared__ double red[4][TILE];

  long long cb;
  int wq;
  if (!xcd_map(n_freq, (Ccols + TILE - 1) / TILE, cb, wq)) return;
  const C *W = Wall + (long long)wq * N * N;
  double *Xout = Xall + (long long)wq * Ccols;
  const long long c0 = cb * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15;
  const int ngroups = (N + TILE - 1) / TILE;
  const int base = N - ngroups * TILE;        // <= 0
  double psum[4] = {0.0, 0.0, 0.0, 0.0};
  // loader mapping: 16 consecutive threads read 16 consecutive nu of one row
  const int lrow = tid >> 4, lk = tid & 15;    // rows lrow + 16*t, t = 0..3

  for (int I = 0; I < ngroups; ++I) {
    const int mu0 = base + I * TILE;
    const int nch = (mu0 + TILE - 2) / SKC + 1;   // chunks covering nu <= mu0 + 62
    const int r0 = mu0 + 16 * wave;               // this wave's first row
    const bool active = (r0 + 15 >= 0);
    const int kcw = active ? (r0 + 14) / SKC + 1 : 0;   // chunks this wave needs (nu <= r0 + 14)
    ACC zr[4], zi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      zr[j] = MF::zero();
      zi[j] = MF::zero();
    }
    C wreg[4], ureg[4];
    auto fetch = [&](int ch) {
      const int nu = ch * SKC + lk;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int m = lrow + 16 * t;
        const int mu = mu0 + m;
        C w;
        w.x = w.y = (T)0;
        if (mu >= 0 && mu < N && nu < mu) w = W[(long long)mu * N + nu];
        wreg[t] = w;
        const long long cc = c0 + m;
        C u;
        u.x = u.y = (T)0;
        if (cc < Ccols && nu < N) u = cconj(x[cc * N + nu]);
        ureg[t] = u;
      }
    };
    auto stash = [&](int b) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        Ws[b][lk][lrow + 16 * t] = wreg[t];
        Us[b][lk][lrow + 16 * t] = ureg[t];
      }
    };
    __syncthreads();
    fetch(0);
    stash(0);
    __syncthreads();
    for (int ch = 0; ch < nch; ++ch) {
      const int b = ch & 1;
      if (ch + 1 < nch) fetch(ch + 1);
      if (ch < kcw) {
#pragma unroll
        for (int ks = 0; ks < SKC / 4; ++ks) {
          const int kk = ks * 4 + (lane >> 4);
          const C a = Ws[b][kk][16 * wave + col];
          C u[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) u[j] = Us[b][kk][16 * j + col];
          // Z += W u: re = Wr ur - Wi ui, im = Wr ui + Wi ur
#pragma unroll
          for (int j = 0; j < 4; ++j) zr[j] = MF::mac(a.x, u[j].x, zr[j]);
#pragma unroll
          for (int j = 0; j < 4; ++j) zi[j] = MF::mac(a.x, u[j].y, zi[j]);
#pragma unroll
          for (int j = 0; j < 4; ++j) zr[j] = MF::mac(-a.y, u[j].y, zr[j]);
#pragma unroll
          for (int j = 0; j < 4; ++j) zi[j] = MF::mac(a.y, u[j].x, zi[j]);
        }
      }
      if (ch + 1 < nch) stash(b ^ 1);
      __syncthreads();
    }
    // epilogue of the group: X_c += 2 Re(x_mu Z_mu) + Re W_mumu |x_mu|^2 over this wave's rows
    if (active) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long long cc = c0 + 16 * j + col;
        if (cc >= Ccols) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int mu = r0 + MF::row(lane, q);
          if (mu < 0 || mu >= N) continue;
          const C xv = x[cc * N + mu];
          const double wdd = (double)W[(long long)mu * N + mu].x;
          const double xr = (double)xv.x, xi = (double)xv.y;
          psum[j] += 2.0 * (xr * (double)zr[j][q] - xi * (double)zi[j][q]) + wdd * (xr * xr + xi * xi);
        }
      }
    }
  }
  // lanes l, l^16, l^32, l^48 hold the same column
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double v = psum[j];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    psum[j] = v;
  }
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave][16 * j + lane] = psum[j];
  }
  __syncthreads();
  if (tid < TILE) {
    const long long cc = c0 + tid;
    if (cc < Ccols) Xout[cc] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  }
}

// Split forms.  conj(x) and the strictly lower part of W^c are split once per
// q into NS 16-bit parts (x = sum_p x_p, each part the rounding of what the
// previous ones left) in zero-padded MFMA-ready arrays:
//   xs[p][re/im][Cpad][Npad]             (Cpad = 64-multiple, Npad = 32-multiple)
//   ws[w][p][re/im][Rpad][Npad]          (row r <-> mu = r + N - Rpad, end-aligned
//                                          64-row groups; zero for nu >= mu)
// Parts are BF16 (H = false) or FP16 (H = true); FP16 parts are taken of the
// values times a power of two, one per x column (sx) and one per frequency of
// W^c (from its largest magnitude, wmax), which the FP64 epilogue undoes
// exactly.  The main kernel streams operands without per-element work: the x
// tile of a workgroup (64 columns x 32 nu) goes to LDS with 16-byte copies,
// double buffered; each wave reads its 16 rows of W straight into MFMA
// registers; products of parts p + q < NS accumulate in FP32 on the 16x16x32
// MFMA.
#define SKB 32
#define SBP 8

// BF16 xs from x (complex FP32 [C][N]); one thread per (column, 8 nu)
template <int NS>
__global__ void k_split_x(const float2 *__restrict__ x, long long C, int N, long long Cpad, int Npad, us16 *__restrict__ xs) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int g8 = Npad / 8;
  if (t >= Cpad * g8) return;
  const long long c = t / g8;
  const int k0 = (int)(t % g8) * 8;
  us16 re[NS][8], im[NS][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int nu = k0 + e;
    const float2 u = cconj(ld_or(x, c * N + nu, c < C && nu < N, mkcf(0.f, 0.f)));
    us16 a[NS], b[NS];
    split_n<NS, false>(u.x, a);
    split_n<NS, false>(u.y, b);
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      re[p][e] = a[p];
      im[p][e] = b[p];
    }
  }
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    *(u32x4 *)(xs + ((long long)(2 * p) * Cpad + c) * Npad + k0) = *(const u32x4 *)re[p];
    *(u32x4 *)(xs + ((long long)(2 * p + 1) * Cpad + c) * Npad + k0) = *(const u32x4 *)im[p];
  }
}

// FP16 xs: one wave per column; the column's largest |Re|, |Im| sets its scale
// sx[c], then the scaled values are split.  Block = 4 columns.
template <int NS>
__global__ __launch_bounds__(256) void k_split_x_h(const float2 *__restrict__ x, long long C, int N, long long Cpad, int Npad,
                                                   us16 *__restrict__ xs, float *__restrict__ sx) {
  const long long c = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= Cpad) return;
  float m = 0.f;
  if (c < C)
    for (int nu = lane; nu < N; nu += 64) {
      const float2 u = x[c * N + nu];
      m = fmaxf(m, fmaxf(fabsf(u.x), fabsf(u.y)));
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  const float inv = inv_pow2_scale(m);
  if (lane == 0) sx[c] = pow2_scale(m);
  for (int k0 = 8 * lane; k0 < Npad; k0 += 512) {
    us16 re[NS][8], im[NS][8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int nu = k0 + e;
      const float2 u = cconj(ld_or(x, c * N + nu, c < C && nu < N, mkcf(0.f, 0.f)));
      us16 a[NS], b[NS];
      split_n<NS, true>(u.x * inv, a);
      split_n<NS, true>(u.y * inv, b);
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        re[p][e] = a[p];
        im[p][e] = b[p];
      }
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      *(u32x4 *)(xs + ((long long)(2 * p) * Cpad + c) * Npad + k0) = *(const u32x4 *)re[p];
      *(u32x4 *)(xs + ((long long)(2 * p + 1) * Cpad + c) * Npad + k0) = *(const u32x4 *)im[p];
    }
  }
}

// out[s] = max(out[s], largest |Re|, |Im| of v[s][0..n_per)) as float bits
// (non-negative floats order like their bit patterns); grid (blocks, sets)
__global__ __launch_bounds__(256) void k_absmax_sets(const float2 *__restrict__ v, long long n_per, unsigned *__restrict__ out) {
  __shared__ float red[4];
  const float2 *p = v + (long long)blockIdx.y * n_per;
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n_per; i += (long long)gridDim.x * 256) {
    const float2 u = p[i];
    m = fmaxf(m, fmaxf(fabsf(u.x), fabsf(u.y)));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    atomicMax(out + blockIdx.y, __float_as_uint(m));
  }
}

// ws from W^c (complex FP32 [n_freq][N][N]); one thread per (w, row, 8 nu)
template <int NS, bool H>
__global__ void k_split_w(const float2 *__restrict__ W, int N, int Npad, int Rpad, int n_freq, const unsigned *__restrict__ wmax,
                          us16 *__restrict__ ws) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int g8 = Npad / 8;
  const long long per = (long long)Rpad * g8;
  if (t >= per * n_freq) return;
  const int w = (int)(t / per);
  const int r = (int)((t % per) / g8);
  const int k0 = (int)(t % g8) * 8;
  const int mu = r + N - Rpad;
  const float inv = H ? inv_pow2_scale(__uint_as_float(wmax[w])) : 1.f;
  us16 re[NS][8], im[NS][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int nu = k0 + e;
    const float2 v = ld_or(W, ((long long)w * N + mu) * N + nu, mu >= 0 && nu < mu, mkcf(0.f, 0.f));
    us16 a[NS], b[NS];
    split_n<NS, H>(v.x * inv, a);
    split_n<NS, H>(v.y * inv, b);
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      re[p][e] = a[p];
      im[p][e] = b[p];
    }
  }
#pragma unroll
  for (int p = 0; p < NS; ++p) {
    const long long o = (((long long)w * NS + p) * 2) * Rpad;
    *(u32x4 *)(ws + ((o + r) * Npad) + k0) = *(const u32x4 *)re[p];
    *(u32x4 *)(ws + ((o + Rpad + r) * Npad) + k0) = *(const u32x4 *)im[p];
  }
}

__device__ inline u32x4 neg_p(u32x4 v) { return v ^ 0x80008000u; }   // both formats keep the sign in bit 15
template <bool H>
__device__ inline float part_f(us16 v) {
  if constexpr (H) return (float)__builtin_bit_cast(_Float16, v);
  else return (float)__builtin_bit_cast(__bf16, v);
}

template <int NS, int SNW, bool PF, int PAD, bool H>
__global__ __launch_bounds__(256) void k_sigma_split(const us16 *__restrict__ xs, const us16 *__restrict__ ws,
                                                     const float2 *__restrict__ x, const float2 *__restrict__ Wall,
                                                     long long Ccols, long long Cpad, int N, int Npad, int Rpad, int n_freq,
                                                     const float *__restrict__ sx, const unsigned *__restrict__ wmax,
                                                     double *__restrict__ Xall) {
  __shared__ __attribute__((aligned(16))) us16 Bs[2][NS * 2][TILE][SKB + PAD];   // [buf][part*2 + re/im][column][nu]
  __shared__ double red[4][SNW * TILE];
  long long cb;
  int wb;
  if (!xcd_map((n_freq + SNW - 1) / SNW, (Ccols + TILE - 1) / TILE, cb, wb)) return;
  const long long c0 = cb * TILE;
  const int w0 = wb * SNW;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, g = lane >> 4;
  const int ngroups = Rpad / TILE;
  const int base = N - Rpad;
  double psum[SNW][4], fw[SNW], fx[4];
#pragma unroll
  for (int v = 0; v < SNW; ++v) {
    fw[v] = H ? (double)pow2_scale(__uint_as_float(wmax[min(w0 + v, n_freq - 1)])) : 1.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) psum[v][j] = 0.0;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) fx[j] = H ? (double)sx[c0 + 16 * j + col] : 1.0;
  // staging map: thread -> (column, 8-nu group) of the 64 x 32 tile
  const int scol = tid >> 2, sk = (tid & 3) * 8;

  for (int I = 0; I < ngroups; ++I) {
    const int mu0 = base + I * TILE;
    const int nch = (mu0 + TILE - 1 > 0) ? (mu0 + TILE - 1 + SKB - 1) / SKB : 0;   // nu < mu0 + 63
    if (nch == 0) continue;
    const int r0 = mu0 + 16 * wave;
    const int kcw = (r0 + 15 > 0) ? (r0 + 15 + SKB - 1) / SKB : 0;                 // nu < r0 + 15
    const int wrow = I * TILE + 16 * wave + col;                                     // stored row of this lane
    f4v zr[SNW][4], zi[SNW][4];
#pragma unroll
    for (int v = 0; v < SNW; ++v)
#pragma unroll
      for (int j = 0; j < 4; ++j) zr[v][j] = zi[v][j] = Mfma<float>::zero();
    u32x4 bpre[NS * 2];
    const us16 *xsrc = xs + (c0 + scol) * Npad + sk;
    __syncthreads();
#pragma unroll
    for (int pr = 0; pr < NS * 2; ++pr) bpre[pr] = *(const u32x4 *)(xsrc + (long long)pr * Cpad * Npad);
#pragma unroll
    for (int pr = 0; pr < NS * 2; ++pr) *(u32x4 *)&Bs[0][pr][scol][sk] = bpre[pr];
    __syncthreads();
    // this wave's 16 rows of W (every frequency of the block), straight into
    // registers, one chunk ahead
    u32x4 acur[SNW][NS * 2], anext[SNW][NS * 2];
    const us16 *wsrc[SNW];
#pragma unroll
    for (int v = 0; v < SNW; ++v) wsrc[v] = ws + ((long long)min(w0 + v, n_freq - 1) * NS * 2 * Rpad + wrow) * Npad + 8 * g;
    if (PF && kcw > 0) {
#pragma unroll
      for (int v = 0; v < SNW; ++v)
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) acur[v][pr] = *(const u32x4 *)(wsrc[v] + (long long)pr * Rpad * Npad);
    }
    for (int ch = 0; ch < nch; ++ch) {
      const int b = ch & 1;
      if (ch + 1 < nch) {
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) bpre[pr] = *(const u32x4 *)(xsrc + (long long)pr * Cpad * Npad + (ch + 1) * SKB);
      }
      if (PF && ch + 1 < kcw) {
#pragma unroll
        for (int v = 0; v < SNW; ++v)
#pragma unroll
          for (int pr = 0; pr < NS * 2; ++pr)
            anext[v][pr] = *(const u32x4 *)(wsrc[v] + (long long)pr * Rpad * Npad + (ch + 1) * SKB);
      }
      if (!PF && ch < kcw) {
#pragma unroll
        for (int v = 0; v < SNW; ++v)
#pragma unroll
          for (int pr = 0; pr < NS * 2; ++pr)
            acur[v][pr] = *(const u32x4 *)(wsrc[v] + (long long)pr * Rpad * Npad + ch * SKB);
      }
      if (ch < kcw) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          u32x4 br[NS], bi[NS];
#pragma unroll
          for (int p = 0; p < NS; ++p) {
            br[p] = *(const u32x4 *)&Bs[b][2 * p][16 * j + col][8 * g];
            bi[p] = *(const u32x4 *)&Bs[b][2 * p + 1][16 * j + col][8 * g];
          }
#pragma unroll
          for (int v = 0; v < SNW; ++v) {
            // Z += W u: re = Wr ur - Wi ui, im = Wr ui + Wi ur
#pragma unroll
            for (int p = 0; p < NS; ++p) {
              const u32x4 ar = acur[v][2 * p], ai = acur[v][2 * p + 1], nai = neg_p(ai);
#pragma unroll
              for (int q = 0; q + p < NS; ++q) {
                zr[v][j] = mfma_p<H>(ar, br[q], zr[v][j]);
                zr[v][j] = mfma_p<H>(nai, bi[q], zr[v][j]);
                zi[v][j] = mfma_p<H>(ar, bi[q], zi[v][j]);
                zi[v][j] = mfma_p<H>(ai, br[q], zi[v][j]);
              }
            }
          }
        }
      }
      if (ch + 1 < nch) {
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) *(u32x4 *)&Bs[b ^ 1][pr][scol][sk] = bpre[pr];
      }
      if (PF && ch + 1 < kcw) {
#pragma unroll
        for (int v = 0; v < SNW; ++v)
#pragma unroll
          for (int pr = 0; pr < NS * 2; ++pr) acur[v][pr] = anext[v][pr];
      }
      __syncthreads();
    }
    // X_c += 2 Re(x_mu Z_mu) + Re W_mumu |x_mu|^2 over this wave's rows
    if (r0 + 15 >= 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long long cc = c0 + 16 * j + col;
        if (cc >= Ccols) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int mu = r0 + Mfma<float>::row(lane, q);
          if (mu < 0 || mu >= N) continue;
          const float2 xv = x[cc * N + mu];
          const double xr = (double)xv.x, xi = (double)xv.y;
#pragma unroll
          for (int v = 0; v < SNW; ++v) {
            if (w0 + v >= n_freq) continue;
            const double wdd = (double)Wall[((long long)(w0 + v) * N + mu) * N + mu].x;
            psum[v][j] += 2.0 * fw[v] * fx[j] * (xr * (double)zr[v][j][q] - xi * (double)zi[v][j][q]) + wdd * (xr * xr + xi * xi);
          }
        }
      }
    }
  }
#pragma unroll
  for (int v = 0; v < SNW; ++v)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      double t = psum[v][j];
      t += __shfl_xor(t, 16);
      t += __shfl_xor(t, 32);
      psum[v][j] = t;
    }
  __syncthreads();
  if (lane < 16) {
#pragma unroll
    for (int v = 0; v < SNW; ++v)
#pragma unroll
      for (int j = 0; j < 4; ++j) red[wave][v * TILE + 16 * j + lane] = psum[v][j];
  }
  __syncthreads();
  if (tid < SNW * TILE) {
    const int v = tid / TILE, cl = tid % TILE;
    const long long cc = c0 + cl;
    if (cc < Ccols && w0 + v < n_freq)
      Xall[(long long)(w0 + v) * Ccols + cc] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
  }
}

// The same contraction with 32 x 32 wave tiles (waves 2 x 2 over the 64 x 64
// workgroup tile, one frequency): per chunk a wave reads half as many x
// fragments from LDS (two column tiles) and twice as many W fragments from
// L2 (two row tiles, one chunk ahead), for the same MFMA work.
template <int NS, bool PF, bool H>
__global__ __launch_bounds__(256) void k_sigma_splitq(const us16 *__restrict__ xs, const us16 *__restrict__ ws,
                                                      const float2 *__restrict__ x, const float2 *__restrict__ Wall,
                                                      long long Ccols, long long Cpad, int N, int Npad, int Rpad, int n_freq,
                                                      const float *__restrict__ sx, const unsigned *__restrict__ wmax,
                                                      double *__restrict__ Xall) {
  __shared__ __attribute__((aligned(16))) us16 Bs[2][NS * 2][TILE][SKB + SBP];
  __shared__ double red[2][TILE];
  long long cb;
  int w;
  if (!xcd_map(n_freq, (Ccols + TILE - 1) / TILE, cb, w)) return;
  const long long c0 = cb * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, g = lane >> 4;
  const int wr = wave >> 1, wc = wave & 1;
  const int ngroups = Rpad / TILE;
  const int base = N - Rpad;
  double psum[2] = {0.0, 0.0}, fx[2];
  const double fw = H ? (double)pow2_scale(__uint_as_float(wmax[w])) : 1.0;
#pragma unroll
  for (int j = 0; j < 2; ++j) fx[j] = H ? (double)sx[c0 + 32 * wc + 16 * j + col] : 1.0;
  const int scol = tid >> 2, sk = (tid & 3) * 8;
  const us16 *xsrc = xs + (c0 + scol) * Npad + sk;
  const long long pst = (long long)Rpad * Npad;

  for (int I = 0; I < ngroups; ++I) {
    const int mu0 = base + I * TILE;
    const int nch = (mu0 + TILE - 1 > 0) ? (mu0 + TILE - 1 + SKB - 1) / SKB : 0;   // nu < mu0 + 63
    if (nch == 0) continue;
    const int r0 = mu0 + 32 * wr;
    const int kcw = (r0 + 31 > 0) ? (r0 + 31 + SKB - 1) / SKB : 0;                 // nu < r0 + 31
    f4v zr[2][2], zi[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) zr[i][j] = zi[i][j] = Mfma<float>::zero();
    u32x4 bpre[NS * 2];
    __syncthreads();
#pragma unroll
    for (int pr = 0; pr < NS * 2; ++pr) bpre[pr] = *(const u32x4 *)(xsrc + (long long)pr * Cpad * Npad);
#pragma unroll
    for (int pr = 0; pr < NS * 2; ++pr) *(u32x4 *)&Bs[0][pr][scol][sk] = bpre[pr];
    __syncthreads();
    const us16 *wsrc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
      wsrc[i] = ws + ((long long)w * NS * 2 * Rpad + I * TILE + 32 * wr + 16 * i + col) * Npad + 8 * g;
    u32x4 acur[2][NS * 2], anext[2][NS * 2];
    if (PF && kcw > 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) acur[i][pr] = *(const u32x4 *)(wsrc[i] + pr * pst);
    }
    for (int ch = 0; ch < nch; ++ch) {
      const int b = ch & 1;
      if (ch + 1 < nch) {
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) bpre[pr] = *(const u32x4 *)(xsrc + (long long)pr * Cpad * Npad + (ch + 1) * SKB);
      }
      if (PF && ch + 1 < kcw) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int pr = 0; pr < NS * 2; ++pr) anext[i][pr] = *(const u32x4 *)(wsrc[i] + pr * pst + (ch + 1) * SKB);
      }
      if (!PF && ch < kcw) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int pr = 0; pr < NS * 2; ++pr) acur[i][pr] = *(const u32x4 *)(wsrc[i] + pr * pst + ch * SKB);
      }
      if (ch < kcw) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          u32x4 br[NS], bi[NS];
#pragma unroll
          for (int p = 0; p < NS; ++p) {
            br[p] = *(const u32x4 *)&Bs[b][2 * p][32 * wc + 16 * j + col][8 * g];
            bi[p] = *(const u32x4 *)&Bs[b][2 * p + 1][32 * wc + 16 * j + col][8 * g];
          }
#pragma unroll
          for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int p = 0; p < NS; ++p) {
              const u32x4 ar = acur[i][2 * p], ai = acur[i][2 * p + 1], nai = neg_p(ai);
#pragma unroll
              for (int q = 0; q + p < NS; ++q) {
                zr[i][j] = mfma_p<H>(ar, br[q], zr[i][j]);
                zr[i][j] = mfma_p<H>(nai, bi[q], zr[i][j]);
                zi[i][j] = mfma_p<H>(ar, bi[q], zi[i][j]);
                zi[i][j] = mfma_p<H>(ai, br[q], zi[i][j]);
              }
            }
          }
        }
      }
      if (ch + 1 < nch) {
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) *(u32x4 *)&Bs[b ^ 1][pr][scol][sk] = bpre[pr];
      }
      if (PF && ch + 1 < kcw) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int pr = 0; pr < NS * 2; ++pr) acur[i][pr] = anext[i][pr];
      }
      __syncthreads();
    }
    if (r0 + 31 >= 0) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const long long cc = c0 + 32 * wc + 16 * j + col;
        if (cc >= Ccols) continue;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int mu = r0 + 16 * i + Mfma<float>::row(lane, q);
            if (mu < 0 || mu >= N) continue;
            const float2 xv = x[cc * N + mu];
            const double xr = (double)xv.x, xi = (double)xv.y;
            const double wdd = (double)Wall[((long long)w * N + mu) * N + mu].x;
            psum[j] += 2.0 * fw * fx[j] * (xr * (double)zr[i][j][q] - xi * (double)zi[i][j][q]) + wdd * (xr * xr + xi * xi);
          }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    double t = psum[j];
    t += __shfl_xor(t, 16);
    t += __shfl_xor(t, 32);
    psum[j] = t;
  }
  __syncthreads();
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 2; ++j) red[wr][32 * wc + 16 * j + lane] = psum[j];
  }
  __syncthreads();
  if (tid < TILE) {
    const long long cc = c0 + tid;
    if (cc < Ccols) Xall[(long long)w * Ccols + cc] = red[0][tid] + red[1][tid];
  }
}

// Resident-tile form (two-part FP16 split, N_aux <= RES_NPAD): one workgroup of NWV
// waves (8: two per SIMD; 4: one per SIMD with the whole register file) per
// (64 columns, set of F frequencies), the set chosen by the XCD the workgroup
// runs on: with S = 8 sets (F <= RES_F) XCD x takes set x; with S = 4 sets and
// eight waves (F <= 8, one wave per frequency at 32 frequencies) XCDs x and
// x + 4 take set x mod 4 and alternate column blocks, so each x tile is loaded
// by four workgroups instead of eight and serves twice the work.  The split x tile of its columns, every nu, is loaded into
// LDS once; then NWV/F' waves (F' = F rounded up to 1, 2 or 4) share each
// frequency, each working through its own list of 32-row tiles (a balanced
// static assignment built on the host) with its W fragments read one chunk
// ahead from L2, with no barrier until the final reduction.  The per-wave sums
// over mu are reduced through LDS in a fixed order.  items[w * (RES_MAXI + 1)]
// = number of tiles of wave w, then the tiles.
#define RES_NPAD 288
#define RES_F 4
#define RES_MAXI 15

// GX: the per-tile sum X_c += 2 Re(x_mu Z_mu) takes x from the FP32 array in
// global memory (L2-resident while the column block is worked on) instead of
// the FP16 parts in LDS: two 16-byte loads and two FMAs per row quadruple
// instead of four 8-byte LDS reads, four conversions and four FMAs.
template <int PAD, bool H, int NWV, bool GX = false>
__global__ __launch_bounds__(64 * NWV) void k_sigma_res(const us16 *__restrict__ xs, const us16 *__restrict__ ws,
                                                   const float2 *__restrict__ x, const float2 *__restrict__ Wall,
                                                   long long Ccols, long long Cpad, int N, int Npad, int Rpad, int n_freq,
                                                   int F, int S, const int *__restrict__ items, const float *__restrict__ sx,
                                                   const unsigned *__restrict__ wmax, double *__restrict__ Xall) {
  __shared__ __attribute__((aligned(16))) us16 Xs[4][TILE][RES_NPAD + PAD];   // [part*2 + re/im][column][nu]
  const int xcd = blockIdx.x & 7;
  const int fs = xcd % S;
  const long long c0 = ((long long)(blockIdx.x >> 3) * (8 / S) + xcd / S) * TILE;
  const int f0 = fs * F;
  if (f0 >= n_freq || c0 >= Ccols) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, g = lane >> 4;
  const int fpad = F <= 1 ? 1 : F <= 2 ? 2 : F <= 4 ? 4 : 8;
  const int wpf = NWV / fpad;               // waves per frequency
  const int fl = wave / wpf;
  const int w = f0 + fl;
  const int g8 = Npad / 8;
  {
    // 4 x 64 rows of g8 <= RES_NPAD/8 16-byte pieces: wave w takes rows
    // w, w + NWV, ..., lane = piece (no index division); all loads of a batch
    // in flight before its LDS stores
    constexpr int ROWS = 4 * TILE / NWV, BATCH = ROWS;
    const bool lact = lane < g8;
#pragma unroll
    for (int r0b = 0; r0b < ROWS; r0b += BATCH) {
      u32x4 v[BATCH];
#pragma unroll
      for (int t = 0; t < BATCH; ++t) {
        const int row = wave + NWV * (r0b + t);   // = part plane * 64 + column
        if (lact) v[t] = *(const u32x4 *)(xs + ((long long)(row >> 6) * Cpad + c0 + (row & 63)) * Npad + 8 * lane);
      }
#pragma unroll
      for (int t = 0; t < BATCH; ++t) {
        const int row = wave + NWV * (r0b + t);
        if (lact) *(u32x4 *)&Xs[row >> 6][row & 63][8 * lane] = v[t];
      }
    }
  }
  __syncthreads();
  const int base = N - Rpad;
  const long long pst = (long long)Rpad * Npad;
  const int *it = items + wave * (RES_MAXI + 1);
  const int nit = (fl < F && w < n_freq) ? it[0] : 0;
  double psum[4] = {0.0, 0.0, 0.0, 0.0};
  float fx[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) fx[j] = H ? sx[c0 + 16 * j + col] : 1.f;
  const float fw = H ? pow2_scale(__uint_as_float(wmax[min(w, n_freq - 1)])) : 1.f;
  for (int idx = 0; idx < nit; ++idx) {
    const int t = it[1 + idx];
    const int r0 = base + 32 * t;
    const int kcw = (r0 + 31 > 0) ? (r0 + 31 + SKB - 1) / SKB : 0;   // nu < r0 + 31
    f4v zr[2][4], zi[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) zr[i][j] = zi[i][j] = Mfma<float>::zero();
    const us16 *wsrc = ws + ((long long)w * 4 * Rpad + 32 * t + col) * Npad + 8 * g;   // row tile i at + 16 i Npad
    // W fragments of chunk ch into a[i][part*2 + re/im]; the chunk index is
    // clamped so that every iteration issues the same loads (the two register
    // sets alternate, so a wait covers only the older set)
    auto load_a = [&](u32x4 (&a)[2][4], int ch) {
      const int cc = min(ch, kcw - 1) * SKB;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int pr = 0; pr < 4; ++pr) a[i][pr] = *(const u32x4 *)(wsrc + pr * pst + 16 * i * Npad + cc);
    };
    auto chunk = [&](const u32x4 (&a)[2][4], int ch) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        u32x4 br[2], bi[2];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
          br[p] = *(const u32x4 *)&Xs[2 * p][16 * j + col][ch * SKB + 8 * g];
          bi[p] = *(const u32x4 *)&Xs[2 * p + 1][16 * j + col][ch * SKB + 8 * g];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          // Z += W u: re = Wr ur - Wi ui, im = Wr ui + Wi ur; parts p + q < 2
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            const u32x4 ar = a[i][2 * p], ai = a[i][2 * p + 1], nai = neg_p(ai);
#pragma unroll
            for (int q = 0; q + p < 2; ++q) {
              zr[i][j] = mfma_p<H>(ar, br[q], zr[i][j]);
              zr[i][j] = mfma_p<H>(nai, bi[q], zr[i][j]);
              zi[i][j] = mfma_p<H>(ar, bi[q], zi[i][j]);
              zi[i][j] = mfma_p<H>(ai, br[q], zi[i][j]);
            }
          }
        }
      }
    };
    if (kcw > 0) {
      // an odd first chunk is taken alone, so the paired loop has no branch
      // (a conditional second half would pull its loads in behind the branch)
      u32x4 a0[2][4], a1[2][4];
      int ch = kcw & 1;
      if (ch) load_a(a1, 0);
      load_a(a0, ch);
      if (ch) chunk(a1, 0);
      // the scheduling barriers keep each prefetch ahead of the chunk it
      // overlaps (the scheduler would otherwise sink the loads to their use)
      for (; ch < kcw; ch += 2) {
        load_a(a1, ch + 1);
        __builtin_amdgcn_sched_barrier(0);
        chunk(a0, ch);
        load_a(a0, ch + 2);
        __builtin_amdgcn_sched_barrier(0);
        chunk(a1, ch + 1);
      }
    }
    // X_c += 2 Re(x_mu Z_mu) over the tile's rows (the diagonal term is
    // already in X, from the exact x), with x_mu from the resident tile (the
    // sum of its parts: the same x as in Z), in units of the column scale; the
    // tile's eight terms per lane are summed in FP32, the tiles in FP64
    // the tile holds conj(x) / sx = xr - i xi' with xi' = -Im(x) / sx
    float tz[4] = {0.f, 0.f, 0.f, 0.f};
    if (GX && (N & 3) == 0) {
      // tz in units of x (not x/sx): Re(x Z') = xr zr - xi zi with Z' the
      // product of the scaled tile; the column scale is applied once below
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int m0 = r0 + 16 * i + 4 * g;
        const bool ok = m0 >= 0;
        const int ma = ok ? m0 : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const long long cc = c0 + 16 * j + col;
          const long long cs = cc < Ccols ? cc : 0;   // padded columns read column 0 (never stored)
          const float4 *px = (const float4 *)(x + cs * N + ma);   // 4 consecutive rows, 32-byte aligned
          const float4 a = px[0], b = px[1];
          const float xr[4] = {a.x, a.z, b.x, b.z}, xi[4] = {a.y, a.w, b.y, b.w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float zrv = ok ? zr[i][j][q] : 0.f, ziv = ok ? zi[i][j][q] : 0.f;
            tz[j] = fmaf(xr[q], zrv, fmaf(-xi[q], ziv, tz[j]));
          }
        }
      }
    } else if ((N & 3) == 0) {
      // a lane's four rows 16 i + 4 (lane / 16) + q are consecutive and, with
      // N = 0 (mod 4), start on a multiple of 4 (tiles end at row N - 1): one
      // 8-byte read per plane; a group above row 0 reads row 0 and adds zero
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int m0 = r0 + 16 * i + 4 * g;
        const bool ok = m0 >= 0;
        const int ma = ok ? m0 : 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int cl = 16 * j + col;
          uint2 pv[4];
#pragma unroll
          for (int pl = 0; pl < 4; ++pl) pv[pl] = *(const uint2 *)&Xs[pl][cl][ma];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float xp[4];
#pragma unroll
            for (int pl = 0; pl < 4; ++pl) {
              const unsigned wv = (q < 2) ? pv[pl].x : pv[pl].y;
              xp[pl] = part_f<H>((us16)((q & 1) ? (wv >> 16) : (wv & 0xffffu)));
            }
            // Re(x Z), each part taken on its own (the FP16 parts enter the
            // FMAs directly, with no separate conversion and sum)
            const float zrv = ok ? zr[i][j][q] : 0.f, ziv = ok ? zi[i][j][q] : 0.f;
            tz[j] = fmaf(xp[3], ziv, fmaf(xp[1], ziv, fmaf(xp[2], zrv, fmaf(xp[0], zrv, tz[j]))));
          }
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int mu = r0 + 16 * i + Mfma<float>::row(lane, q);
          if (mu < 0 || mu >= N) continue;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int cl = 16 * j + col;
            const float xr = part_f<H>(Xs[0][cl][mu]) + part_f<H>(Xs[2][cl][mu]);
            const float xc = part_f<H>(Xs[1][cl][mu]) + part_f<H>(Xs[3][cl][mu]);
            tz[j] = fmaf(xr, zr[i][j][q], fmaf(xc, zi[i][j][q], tz[j]));   // Re(x Z)
          }
        }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) psum[j] += 2.0 * (double)fw * (double)tz[j];
  }
  // x = sx x' and Z = sW sx Z': sx^2 (sx once when the sum took x itself)
#pragma unroll
  for (int j = 0; j < 4; ++j) psum[j] *= (GX && (N & 3) == 0) ? (double)fx[j] : (double)fx[j] * (double)fx[j];
  // lanes l, l^16, l^32, l^48 hold the same column
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double v = psum[j];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    psum[j] = v;
  }
  __syncthreads();   // the x tile is no longer read: its space takes the partial sums
  double *red = (double *)&Xs[0][0][0];   // [wave][column]
  if (lane < 16) {
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave * TILE + 16 * j + lane] = psum[j];
  }
  __syncthreads();
  const int nf = min(F, n_freq - f0);
  if (tid < nf * TILE) {
    const int f = tid / TILE, cl = tid % TILE;
    double sum = 0.0;
    for (int v = 0; v < wpf; ++v) sum += red[(f * wpf + v) * TILE + cl];
    const long long cc = c0 + cl;
    if (cc < Ccols) Xall[(long long)(f0 + f) * Ccols + cc] += sum;
  }
}

// The diagonal term of the pair weights, exactly: X[w][c] = sum_mu Re W^c_mumu(w)
// |x_c^mu|^2 in FP64 from the FP32 x, for the resident-tile form (which adds
// the off-diagonal part).  wd[mu][w] = Re W^c_mumu(w) (RES_WMAX frequencies
// per row, zero beyond n_freq); one thread per column c.
#define RES_WMAX 32
__global__ void k_wdiag(const float2 *__restrict__ W, int N, int n_freq, double *__restrict__ wd) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * RES_WMAX) return;
  const int mu = t / RES_WMAX, w = t % RES_WMAX;
  wd[t] = w < n_freq ? (double)W[((long long)w * N + mu) * N + mu].x : 0.0;
}
// D[w][c] = sum_mu Re W^c_mumu(w) |x_mu(c)|^2 as an FP64 matrix product on the
// 16x16x4 MFMA (A = W^c_mumu, 16 frequencies x 4 mu; B = |x|^2, 4 mu x 16
// columns): a workgroup takes 64 columns, each wave 16 of them and all
// RES_WMAX frequencies (two accumulators).  The x rows of the 64 columns are
// read in 64-mu chunks, one row's chunk (512 contiguous bytes) per wave-wide
// load, and |x|^2 (FP64) and the chunk's W^c diagonal go through LDS into
// the operand layouts: in the j-th product of a chunk lane l holds
// mu = m0 + 4 j + l / 16 for frequency l % 16 (A) and column l % 16 (B).
// Entries past N or C are zero.
static_assert(RES_WMAX == 32, "two 16-frequency accumulators");
__global__ __launch_bounds__(256) void k_pair_diag(const float2 *__restrict__ x, long long C, int N, int n_freq,
                                                   const double *__restrict__ wd, double *__restrict__ Xall) {
  __shared__ double a2s[64][64 + 1];          // [mu - m0][column - c0]
  __shared__ double wds[64][RES_WMAX + 1];    // [mu - m0][frequency]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long long c0 = (long long)blockIdx.x * 64;
  Mfma<double>::acc a0 = Mfma<double>::zero(), a1 = Mfma<double>::zero();
  for (int m0 = 0; m0 < N; m0 += 64) {
    const int mu = m0 + lane;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const long long cr = c0 + 16 * wave + r;
      v[r] = ld_or(x, cr * N + mu, cr < C && mu < N, mkcf(0.f, 0.f));
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) a2s[lane][16 * wave + r] = (double)v[r].x * (double)v[r].x + (double)v[r].y * (double)v[r].y;
#pragma unroll
    for (int i = 0; i < 64 * RES_WMAX / 256; ++i) {
      const int e = tid + 256 * i, m = e / RES_WMAX, w = e % RES_WMAX;
      wds[m][w] = ld_or(wd, (long long)(m0 + m) * RES_WMAX + w, m0 + m < N, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      if (m0 + 4 * j >= N) break;   // the rest of the chunk lies past N (same for the whole workgroup)
      const int m = 4 * j + (lane >> 4);
      const double b = a2s[m][16 * wave + (lane & 15)];
      a0 = Mfma<double>::mac(wds[m][lane & 15], b, a0);
      a1 = Mfma<double>::mac(wds[m][16 + (lane & 15)], b, a1);
    }
    __syncthreads();
  }
  const long long c = c0 + 16 * wave + (lane & 15);
  if (c >= C) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int w = Mfma<double>::row(lane, r);
    if (w < n_freq) Xall[(long long)w * C + c] = a0[r];
    if (16 + w < n_freq) Xall[(long long)(16 + w) * C + c] = a1[r];
  }
}

// Tile lists of the resident-tile form: the 32-row tiles with work are shared
// by the NWV/F' waves of a frequency, largest first to the least loaded wave
// (cost = number of nu chunks); every frequency slot gets the same lists.
// With eight waves, waves w and w + 4 share a SIMD (waves are placed on the
// SIMDs in turn) and their MFMA pipe: the second four take the lists in the
// opposite order, so that each SIMD runs a heavier and a lighter list.
static bool sigma_res_plan(int N, int n_freq, int NWV, int sets, std::vector<int> &table, int &F) {
  const int Npad = (N + SKB - 1) / SKB * SKB, Rpad = (N + TILE - 1) / TILE * TILE;
  F = (n_freq + sets - 1) / sets;
  if (Npad > RES_NPAD || F > (sets == 8 ? RES_F : NWV)) return false;
  const int fpad = F <= 1 ? 1 : F <= 2 ? 2 : F <= 4 ? 4 : 8;
  const int wpf = NWV / fpad;
  const int base = N - Rpad;
  std::vector<std::pair<int, int>> its;   // (cost, tile)
  for (int t = 0; t < Rpad / 32; ++t) {
    const int r0 = base + 32 * t;
    const int kcw = (r0 + 31 > 0) ? (r0 + 31 + SKB - 1) / SKB : 0;
    if (kcw > 0) its.push_back({kcw, t});
  }
  std::stable_sort(its.begin(), its.end(), [](const std::pair<int, int> &a, const std::pair<int, int> &b) { return a.first > b.first; });
  std::vector<std::vector<int>> lists(wpf);
  std::vector<int> load(wpf, 0);
  for (const auto &pr : its) {
    int wv = 0;
    for (int v = 1; v < wpf; ++v)
      if (load[v] < load[wv]) wv = v;
    load[wv] += pr.first;
    lists[wv].push_back(pr.second);
  }
  // heaviest list first
  std::vector<int> order(wpf);
  for (int v = 0; v < wpf; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load[a] > load[b]; });
  table.assign(NWV * (RES_MAXI + 1), 0);
  for (int wave = 0; wave < NWV; ++wave) {
    int li = wave % wpf;
    if (NWV == 8 && wave >= 4) li = wpf <= 4 ? wpf - 1 - li : 11 - wave;
    const std::vector<int> &l = lists[order[li]];
    if ((int)l.size() > RES_MAXI) return false;
    table[wave * (RES_MAXI + 1)] = (int)l.size();
    for (size_t i = 0; i < l.size(); ++i) table[wave * (RES_MAXI + 1) + 1 + i] = l[i];
  }
  return true;
}

int sigma_res_prepare(lrigw_ctx *c) {
  c->sig_res_ok = false;
  // the epilogue takes x from the split tile: 22 significand bits with FP16
  // parts, too few with BF16 ones
  if (ns_sig(c->precision) != 2 || !split_h(c->precision)) return LRIGW_OK;
  std::vector<int> t8, t4, t84;
  int F = 0, F4 = 0;
  if (c->d.n_freq > RES_WMAX) return LRIGW_OK;
  if (!sigma_res_plan(c->d.n_aux, c->d.n_freq, 8, 8, t8, F) || !sigma_res_plan(c->d.n_aux, c->d.n_freq, 4, 8, t4, F))
    return LRIGW_OK;
  if (!sigma_res_plan(c->d.n_aux, c->d.n_freq, 8, 4, t84, F4)) t84.assign(8 * (RES_MAXI + 1), 0), F4 = 0;
  LRIGW_HIP_TRY(hipMalloc(&c->d_wd, (size_t)c->d.n_aux * RES_WMAX * sizeof(double)));
  // the 8-wave lists, the 4-wave ones, then the 8-wave lists of four sets
  t8.insert(t8.end(), t4.begin(), t4.end());
  t8.insert(t8.end(), t84.begin(), t84.end());
  LRIGW_HIP_TRY(hipMalloc(&c->d_sitems, t8.size() * sizeof(int)));
  LRIGW_HIP_TRY(hipMemcpy(c->d_sitems, t8.data(), t8.size() * sizeof(int), hipMemcpyHostToDevice));
  c->sig_res_F = F;
  c->sig_res_F4 = F4;
  c->sig_res_ok = true;
  return LRIGW_OK;
}

// the same lists for a second plane count (the real-axis planes of contour
// deformation); without them those planes run in the tuner-free split form
int sigma_res_prepare_real(lrigw_ctx *c, int n_r) {
  c->sig_res_nr = 0;
  if (!c->sig_res_ok || n_r > RES_WMAX) return LRIGW_OK;
  std::vector<int> t8, t4, t84;
  int F = 0, F4 = 0;
  if (!sigma_res_plan(c->d.n_aux, n_r, 8, 8, t8, F) || !sigma_res_plan(c->d.n_aux, n_r, 4, 8, t4, F)) return LRIGW_OK;
  if (!sigma_res_plan(c->d.n_aux, n_r, 8, 4, t84, F4)) t84.assign(8 * (RES_MAXI + 1), 0), F4 = 0;
  t8.insert(t8.end(), t4.begin(), t4.end());
  t8.insert(t8.end(), t84.begin(), t84.end());
  if (!c->d_sitems_r) LRIGW_HIP_TRY(hipMalloc(&c->d_sitems_r, t8.size() * sizeof(int)));   // fixed size per cell
  LRIGW_HIP_TRY(hipMemcpy(c->d_sitems_r, t8.data(), t8.size() * sizeof(int), hipMemcpyHostToDevice));
  c->sig_res_Fr = F;
  c->sig_res_Fr4 = F4;
  c->sig_res_nr = n_r;
  return LRIGW_OK;
}

// sigma[k][n][i] += scale * sum_m sum_j g_j X[j][k][n][m] a/(a^2 + w_j^2),  a = i w_i + mu - e_m(k-q)
// One wave per (k, SF_I frequencies i, SF_N bands n): lanes run over the pairs
// (m, j), m fastest (coalesced X), so each kernel value g_j a/(a^2 + w_j^2) is
// formed once and serves every n; the lane sums are reduced through LDS in a
// fixed order (one output per lane).
#define SF_I 4
#define SF_N 8
__global__ __launch_bounds__(64) void k_sigma_freq(const double *__restrict__ X, const double *__restrict__ eig,
                                                   const int *__restrict__ kmq, int iq, int nk, int n_qp, int n_bands,
                                                   int n_freq, const double *__restrict__ omega, const double *__restrict__ weight,
                                                   double mu, double scale, double2 *__restrict__ sigma) {
  __shared__ double red[2 * SF_I * SF_N][65];
  const int k = blockIdx.x, i0 = blockIdx.y * SF_I, n0 = blockIdx.z * SF_N, lane = threadIdx.x;
  const int k2 = kmq[k * nk + iq];
  const long long cstride = (long long)nk * n_qp * n_bands;
  double wi[SF_I];
#pragma unroll
  for (int ii = 0; ii < SF_I; ++ii) wi[ii] = i0 + ii < n_freq ? omega[i0 + ii] : 1.0;
  double accr[SF_I][SF_N], acci[SF_I][SF_N];
#pragma unroll
  for (int ii = 0; ii < SF_I; ++ii)
#pragma unroll
    for (int n = 0; n < SF_N; ++n) accr[ii][n] = acci[ii][n] = 0.0;
  const int np = n_bands * n_freq;
  for (int p = lane; p < np; p += 64) {
    const int j = p / n_bands, m = p % n_bands;
    const double ar = mu - eig[(long long)k2 * n_bands + m];
    const double wj = omega[j], gj = weight[j];
    const double *xp = X + (long long)j * cstride + ((long long)k * n_qp + n0) * n_bands + m;
    double x[SF_N];
#pragma unroll
    for (int n = 0; n < SF_N; ++n) x[n] = gj * ld_or(xp, (long long)n * n_bands, n0 + n < n_qp, 0.0);
#pragma unroll
    for (int ii = 0; ii < SF_I; ++ii) {
      const double ai = wi[ii];
      const double dr = ar * ar - ai * ai + wj * wj, di = 2.0 * ar * ai;
      const double inv = 1.0 / (dr * dr + di * di);
      const double kr = (ar * dr + ai * di) * inv, ki = (ai * dr - ar * di) * inv;
#pragma unroll
      for (int n = 0; n < SF_N; ++n) {
        accr[ii][n] += x[n] * kr;
        acci[ii][n] += x[n] * ki;
      }
    }
  }
#pragma unroll
  for (int ii = 0; ii < SF_I; ++ii)
#pragma unroll
    for (int n = 0; n < SF_N; ++n) {
      red[2 * (ii * SF_N + n)][lane] = accr[ii][n];
      red[2 * (ii * SF_N + n) + 1][lane] = acci[ii][n];
    }
  __syncthreads();
  if (lane >= SF_I * SF_N) return;
  const int ii = lane / SF_N, n = lane % SF_N;   // one output per lane
  double sr = 0.0, si = 0.0;
  for (int l = 0; l < 64; ++l) {
    sr += red[2 * lane][l];
    si += red[2 * lane + 1][l];
  }
  if (i0 + ii < n_freq && n0 + n < n_qp) {
    const long long o = ((long long)k * n_qp + n0 + n) * n_freq + i0 + ii;
    double2 s = sigma[o];
    s.x += scale * sr;
    s.y += scale * si;
    sigma[o] = s;
  }
}

// split kernel variants the tuner chooses from: (frequencies per workgroup,
// W prefetched one chunk ahead, wave tile) = (1, yes, 16x64), (2, no, 16x64),
// (1, no, 16x64), (1, yes, 32x32), (1, no, 32x32), the first one with LDS rows
// padded to 96 and 112 bytes instead of 80, and the resident-tile form with 8
// and 4 waves per workgroup and LDS rows padded by 8 or 16 elements, 11/12 the
// 8/4-wave forms whose per-tile sum reads x from global memory (two-part FP16
// split, N_aux <= 288 only)
#define SIGMA_VARIANTS 14
int sigma_variant_snw(int var) { return var == 1 ? 2 : 1; }
int sigma_variants() { return SIGMA_VARIANTS; }
int sigma_default_variant(int precision) { return ns_sig(precision) == 2 ? 1 : 0; }
bool sigma_variant_ok(const lrigw_ctx *c, int var) {
  if (var < 0 || var >= SIGMA_VARIANTS) return false;
  return var < 7 || (c->sig_res_ok && (var != 13 || c->sig_res_F4 > 0));
}

template <int NS, bool H>
static void launch_sigma_split(int var, dim3 gs, hipStream_t st, const us16 *xs, const us16 *ws, const float2 *x,
                               const float2 *W, long long Ccols, long long Cpad, int N, int Npad, int Rpad, int n_freq,
                               const float *sx, const unsigned *wmax, double *X) {
#define SIG_ARGS xs, ws, x, W, Ccols, Cpad, N, Npad, Rpad, n_freq, sx, wmax, X
  switch (var) {
    case 0: hipLaunchKernelGGL((k_sigma_split<NS, 1, true, SBP, H>), gs, dim3(256), 0, st, SIG_ARGS); break;
    case 1: hipLaunchKernelGGL((k_sigma_split<NS, 2, false, SBP, H>), gs, dim3(256), 0, st, SIG_ARGS); break;
    case 2: hipLaunchKernelGGL((k_sigma_split<NS, 1, false, SBP, H>), gs, dim3(256), 0, st, SIG_ARGS); break;
    case 3: hipLaunchKernelGGL((k_sigma_splitq<NS, true, H>), gs, dim3(256), 0, st, SIG_ARGS); break;
    case 4: hipLaunchKernelGGL((k_sigma_splitq<NS, false, H>), gs, dim3(256), 0, st, SIG_ARGS); break;
    case 5: hipLaunchKernelGGL((k_sigma_split<NS, 1, true, 16, H>), gs, dim3(256), 0, st, SIG_ARGS); break;
    default: hipLaunchKernelGGL((k_sigma_split<NS, 1, true, 24, H>), gs, dim3(256), 0, st, SIG_ARGS); break;
  }
#undef SIG_ARGS
}

// X[j][k][n][m] = Re x_nm^T W^c(w_j) conj(x_nm) for the first nw <= N_w
// planes of Wc (the split workspaces hold N_w)
int run_pair_weights(lrigw_ctx *c, const void *x, const void *Wc, int nw, double *X) {
  const Dims &d = c->d;
  const long long Ccols = (long long)d.n_k * d.n_qp * d.n_bands;
  hipEvent_t ev;
  stage_begin(c, "sigma_mfma", &ev);
  const long long ncb = (Ccols + TILE - 1) / TILE;
  dim3 grid(xcd_grid(nw, ncb));
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_sigma_mfma<double>, grid, dim3(256), 0, c->stream, (const double2 *)x, (const double2 *)Wc, Ccols,
                       d.n_aux, nw, X);
  else if (c->precision == LRIGW_FP32)
    hipLaunchKernelGGL(k_sigma_mfma<float>, grid, dim3(256), 0, c->stream, (const float2 *)x, (const float2 *)Wc, Ccols,
                       d.n_aux, nw, X);
  else {
    const long long Cpad = (Ccols + TILE - 1) / TILE * TILE;
    const int Npad = (d.n_aux + SKB - 1) / SKB * SKB;
    const int Rpad = (d.n_aux + TILE - 1) / TILE * TILE;
    us16 *xs = (us16 *)c->d_xs, *ws = (us16 *)c->d_ws;
    const long long nx = Cpad * (Npad / 8), nwt = (long long)nw * Rpad * (Npad / 8);
    const int NS = ns_sig(c->precision);
    const bool H = split_h(c->precision);
    const float2 *xf = (const float2 *)x, *Wf = (const float2 *)Wc;
    const dim3 gx((unsigned)((nx + 255) / 256)), gw((unsigned)((nwt + 255) / 256));
    if (H) {
      // per-frequency largest |W^c| for the FP16 scales
      LRIGW_TRY(zero_fill(c->stream, c->d_wmax, (size_t)nw * sizeof(unsigned)));
      const long long nn = (long long)d.n_aux * d.n_aux;
      const unsigned nb = (unsigned)std::min<long long>((nn + 4095) / 4096, 64);
      hipLaunchKernelGGL(k_absmax_sets, dim3(nb, nw), dim3(256), 0, c->stream, Wf, nn, c->d_wmax);
      hipLaunchKernelGGL(k_split_x_h<2>, dim3((unsigned)(Cpad / 4)), dim3(256), 0, c->stream, xf, Ccols, d.n_aux, Cpad, Npad,
                         xs, c->d_sx);
      hipLaunchKernelGGL((k_split_w<2, true>), gw, dim3(256), 0, c->stream, Wf, d.n_aux, Npad, Rpad, nw, c->d_wmax, ws);
    } else if (NS == 2) {
      hipLaunchKernelGGL(k_split_x<2>, gx, dim3(256), 0, c->stream, xf, Ccols, d.n_aux, Cpad, Npad, xs);
      hipLaunchKernelGGL((k_split_w<2, false>), gw, dim3(256), 0, c->stream, Wf, d.n_aux, Npad, Rpad, nw, nullptr, ws);
    } else {
      hipLaunchKernelGGL(k_split_x<3>, gx, dim3(256), 0, c->stream, xf, Ccols, d.n_aux, Cpad, Npad, xs);
      hipLaunchKernelGGL((k_split_w<3, false>), gw, dim3(256), 0, c->stream, Wf, d.n_aux, Npad, Rpad, nw, nullptr, ws);
    }
    // the resident-tile form has plans for the N_w imaginary planes and for
    // the real-axis grid; any other plane count takes the default split form
    const bool plan_w = nw == d.n_freq, plan_r = !plan_w && nw == c->sig_res_nr;
    int var = (c->sig_var >= 7 && !plan_w && !plan_r) ? sigma_default_variant(c->precision) : c->sig_var;
    const int *items = plan_w ? c->d_sitems : c->d_sitems_r;
    int Fres = plan_w ? c->sig_res_F : c->sig_res_Fr;
    const int F4 = plan_w ? c->sig_res_F4 : c->sig_res_Fr4;
    if (var == 13 && F4 == 0) var = 7;   // no four-set plan for these planes
    if (var >= 7) {
      if (!c->sig_res_ok) return LRIGW_ERR_ARG;
      // the exact diagonal term first; the resident kernel adds the rest
      hipLaunchKernelGGL(k_wdiag, dim3((unsigned)((d.n_aux * RES_WMAX + 255) / 256)), dim3(256), 0, c->stream, Wf, d.n_aux,
                         nw, c->d_wd);
      hipLaunchKernelGGL(k_pair_diag, dim3((unsigned)((Ccols + 63) / 64)), dim3(256), 0, c->stream, xf, Ccols, d.n_aux,
                         nw, c->d_wd, X);
    }
    stage_end(c, "sigma_split", ev);
    stage_begin(c, "sigma_mfma", &ev);
    const int snw = sigma_variant_snw(var);
    dim3 gs(xcd_grid((nw + snw - 1) / snw, ncb));
    if (var >= 7) {
      const dim3 gr((unsigned)(8 * ncb));
      const int *t8 = items, *t4 = items + 8 * (RES_MAXI + 1), *t84 = items + 12 * (RES_MAXI + 1);
#define RES_ARGS xs, ws, xf, Wf, Ccols, Cpad, d.n_aux, Npad, Rpad, nw, Fres, 8
      if (var == 7) hipLaunchKernelGGL((k_sigma_res<8, true, 8>), gr, dim3(512), 0, c->stream, RES_ARGS, t8, c->d_sx, c->d_wmax, X);
      else if (var == 8) hipLaunchKernelGGL((k_sigma_res<8, true, 4>), gr, dim3(256), 0, c->stream, RES_ARGS, t4, c->d_sx, c->d_wmax, X);
      else if (var == 9) hipLaunchKernelGGL((k_sigma_res<16, true, 8>), gr, dim3(512), 0, c->stream, RES_ARGS, t8, c->d_sx, c->d_wmax, X);
      else if (var == 10) hipLaunchKernelGGL((k_sigma_res<16, true, 4>), gr, dim3(256), 0, c->stream, RES_ARGS, t4, c->d_sx, c->d_wmax, X);
      else if (var == 11) hipLaunchKernelGGL((k_sigma_res<8, true, 8, true>), gr, dim3(512), 0, c->stream, RES_ARGS, t8, c->d_sx, c->d_wmax, X);
      else if (var == 12) hipLaunchKernelGGL((k_sigma_res<8, true, 4, true>), gr, dim3(256), 0, c->stream, RES_ARGS, t4, c->d_sx, c->d_wmax, X);
#undef RES_ARGS
      else
        hipLaunchKernelGGL((k_sigma_res<8, true, 8>), dim3((unsigned)(8 * ((ncb + 1) / 2))), dim3(512), 0, c->stream, xs, ws,
                           xf, Wf, Ccols, Cpad, d.n_aux, Npad, Rpad, nw, F4, 4, t84, c->d_sx, c->d_wmax, X);
    } else if (H)
      launch_sigma_split<2, true>(var, gs, c->stream, xs, ws, xf, Wf, Ccols, Cpad, d.n_aux, Npad, Rpad, nw, c->d_sx,
                                  c->d_wmax, X);
    else if (NS == 2)
      launch_sigma_split<2, false>(var, gs, c->stream, xs, ws, xf, Wf, Ccols, Cpad, d.n_aux, Npad, Rpad, nw, nullptr,
                                   nullptr, X);
    else
      launch_sigma_split<3, false>(var, gs, c->stream, xs, ws, xf, Wf, Ccols, Cpad, d.n_aux, Npad, Rpad, nw, nullptr,
                                   nullptr, X);
  }
  stage_end(c, "sigma_mfma", ev);
  LRIGW_TRY(lrigw_launch_check("sigma_mfma"));
  return LRIGW_OK;
}

int run_sigma_c(lrigw_ctx *c, int iq, const void *x, const void *Wc, const double *eig, void *sigma_acc) {
  const Dims &d = c->d;
  hipEvent_t ev_all;
  stage_begin(c, "sigma_c", &ev_all);
  LRIGW_TRY(run_pair_weights(c, x, Wc, d.n_freq, (double *)c->d_X));
  dim3 g2((unsigned)d.n_k, (unsigned)((d.n_freq + SF_I - 1) / SF_I), (unsigned)((d.n_qp + SF_N - 1) / SF_N));
  const double scale = -1.0 / (M_PI * d.n_k);
  hipLaunchKernelGGL(k_sigma_freq, g2, dim3(64), 0, c->stream, (const double *)c->d_X, eig, c->d_kmq, iq, d.n_k, d.n_qp,
                     d.n_bands, d.n_freq, c->d_omega, c->d_weight, d.mu, scale, (double2 *)sigma_acc);
  LRIGW_TRY(lrigw_launch_check("sigma_freq"));
  stage_end(c, "sigma_c", ev_all);
  return LRIGW_OK;
}
