// Independent-particle response on the auxiliary basis (Eq. chi0_matrix):
//   chi~(q, i w)[mu][nu] = -(2/N_k) sum_K 2 D_K/(D_K^2 + w^2) B[K][mu] conj(B[K][nu])
// as a weighted Hermitian rank-K update on MFMA.  Only lower 64x64 tiles are
// computed; the K range is split over workgroups and the partial tiles are
// summed in FP64 in a fixed order (deterministic); the weights are applied to
// the B-side operand in registers, NW frequencies share every LDS tile.
#include <algorithm>
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

#define KC 16          // K rows staged in LDS per step
#define KSUB 1024      // FP32: K rows accumulated by MFMA before flushing into the second-level sum

int launch_delta(lrigw_ctx *c, int iq, const double *eig);
int launch_gamma_modify(lrigw_ctx *c, const void *B);

__device__ inline void tri_decode(int t, int &I, int &J) {
  int i = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  I = i;
  J = t - i * (i + 1) / 2;
}

template <typename T> struct Chi0Cfg;
template <> struct Chi0Cfg<float> { static const int NW = 4; static const bool two_level = true; };
template <> struct Chi0Cfg<double> { static const int NW = 2; static const bool two_level = false; };

// frequencies per workgroup: the default and the alternative the tuner may pick
int chi0_default_nw(int precision) { return precision == LRIGW_FP64 ? Chi0Cfg<double>::NW : Chi0Cfg<float>::NW; }
int chi0_alt_nw(int precision) { return precision == LRIGW_FP64 ? 1 : 2; }

// Complex-frequency planes (cpltab != nullptr): plane w holds, for
// z^2 = -om2 + i s (z = w_r + i eta: om2 = eta^2 - w_r^2, s = 2 w_r eta), the real
// (cpltab[w].y == 0) or imaginary part of the weight 2D/(D^2 - z^2):
//   2D a/(a^2 + s^2)  or  2D s/(a^2 + s^2),  a = D^2 + om2,   s = cpltab[w].x;
// the response at z is then the Re plane plus i times the Im plane.
template <typename T, int NW>
__global__ __launch_bounds__(256) void k_chi0_mfma(const typename c2t<T>::type *__restrict__ B, const T *__restrict__ delta,
                                                   const double *__restrict__ om2tab, const double2 *__restrict__ cpltab,
                                                   const int *__restrict__ wsel,
                                                   const int *__restrict__ run, long long K, int N, int n_freq, long long Ks,
                                                   long long ntile, typename c2t<T>::type *__restrict__ part) {
  if (run && *run == 0) return;
  typedef typename c2t<T>::type C;
  typedef Mfma<T> MF;
  typedef typename MF::acc ACC;
  __shared__ C As[KC][TILE];
  __shared__ C Bs[KC][TILE];
  __shared__ T dl[KC];

  int I, J;
  tri_decode(blockIdx.x, I, J);
  const int w0 = blockIdx.y * NW;
  const long long kb = (long long)blockIdx.z * Ks;
  const long long ke = min(K, kb + Ks);
  const int mu0 = I * TILE, nu0 = J * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, col = lane & 15;

  T om2[NW], csv[NW];
  bool cim[NW];
  const bool cplx = cpltab != nullptr;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const bool in = w0 + w < n_freq;
    om2[w] = (T)(in ? om2tab[wsel[w0 + w]] : 0.0);
    const double2 cp = (cplx && in) ? cpltab[wsel[w0 + w]] : mkc(0.0, 0.0);
    csv[w] = (T)cp.x;
    cim[w] = cp.y != 0.0;
  }
  ACC re[NW][2][2], im[NW][2][2];
  ACC re2[NW][2][2], im2[NW][2][2];
#pragma unroll
  for (int w = 0; w < NW; ++w)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) {
        re[w][si][sj] = MF::zero();
        im[w][si][sj] = MF::zero();
        re2[w][si][sj] = MF::zero();
        im2[w][si][sj] = MF::zero();
      }

  int step = 0;
  for (long long k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int t = 0; t < (KC * TILE) / 256; ++t) {
      int e = tid + 256 * t;
      int kk = e / TILE, m = e % TILE;
      long long kr = k0 + kk;
      C za;
      za.x = za.y = (T)0;
      C a = za, b = za;
      if (kr < ke) {
        if (mu0 + m < N) a = B[kr * N + mu0 + m];
        if (nu0 + m < N) b = B[kr * N + nu0 + m];
      }
      As[kk][m] = a;
      Bs[kk][m] = b;
    }
    if (tid < KC) dl[tid] = (k0 + tid < ke) ? delta[k0 + tid] : (T)1;
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      C av[2], bv[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        av[s] = As[kk][32 * wr + 16 * s + col];
        bv[s] = Bs[kk][32 * wc + 16 * s + col];
      }
      const T d = dl[kk];
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        T wt;
        if (cplx) {
          const T a = d * d + om2[w];
          wt = (T)2 * d * (cim[w] ? csv[w] : a) / (a * a + csv[w] * csv[w]);
        } else {
          wt = (T)2 * d / (d * d + om2[w]);
        }
#pragma unroll
        for (int sj = 0; sj < 2; ++sj) {
          const T br = wt * bv[sj].x, bi = wt * bv[sj].y;
#pragma unroll
          for (int si = 0; si < 2; ++si) {
            // a conj(b) = (ar br + ai bi) + i (ai br - ar bi)
            re[w][si][sj] = MF::mac(av[si].x, br, re[w][si][sj]);
            re[w][si][sj] = MF::mac(av[si].y, bi, re[w][si][sj]);
            im[w][si][sj] = MF::mac(av[si].y, br, im[w][si][sj]);
            im[w][si][sj] = MF::mac(-av[si].x, bi, im[w][si][sj]);
          }
        }
      }
    }
    __syncthreads();
    if (Chi0Cfg<T>::two_level && ++step == KSUB / KC) {
      step = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w)
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
          for (int sj = 0; sj < 2; ++sj) {
            re2[w][si][sj] += re[w][si][sj];
            im2[w][si][sj] += im[w][si][sj];
            re[w][si][sj] = MF::zero();
            im[w][si][sj] = MF::zero();
          }
    }
  }
  const int nfo = (int)n_freq;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w0 + w >= nfo) continue;
    C *dst = part + (((long long)blockIdx.z * n_freq + w0 + w) * ntile + blockIdx.x) * (TILE * TILE);
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) {
        ACC r = re[w][si][sj], i = im[w][si][sj];
        if (Chi0Cfg<T>::two_level) {
          r += re2[w][si][sj];
          i += im2[w][si][sj];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int row = 32 * wr + 16 * si + MF::row(lane, q);
          int cl = 32 * wc + 16 * sj + col;
          C z;
          z.x = r[q];
          z.y = i[q];
          dst[row * TILE + cl] = z;
        }
      }
  }
}

// Split-BF16 form of the same update: every FP32 operand is split into NS
// BF16 parts (x = x_0 + x_1 [+ x_2], x_p = bf16(x - x_0 - ... - x_{p-1})) and
// the products x_p y_q with p + q < NS are accumulated by the 16x16x32 BF16
// MFMA in FP32 (NS = 2: hi*hi + hi*lo + lo*hi; NS = 3: six products, FP32-like
// accuracy).  The unweighted side is split once per LDS tile; the weighted
// side is kept in FP32 in LDS and weighted and split per frequency in
// registers.  The split-K chunks are kept short (<= 2048 rows by default, see
// chi0_plan_splits; the tuner and lrigw_set_tiles allow at most
// CHI0_SPLIT_MAX_ROWS) so that FP32 accumulation error stays ~1e-6.
#define KCB 32
#define BAP 8    // bf16 padding of an A row in LDS
#define BBP 2    // complex padding of a B row in LDS

template <int NS>
__device__ inline void splitn(float v, __bf16 *p) {
  float r = v;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    p[i] = (__bf16)r;
    r -= (float)p[i];
  }
}

// Split-BF16 form.  Once per q the response operand B[K][N] is rewritten as
//   Ap[p][re/im][Npad][Kp]  BF16 parts (row mu, k contiguous, zero padded)
//   Bt[Npad][Kp]            the FP32 values transposed (row nu, k contiguous)
// (Npad: 64-multiple, Kp: 32-multiple).  In the main kernel a workgroup owns a
// 64 x 64 tile (rows mu, columns nu), each wave a 64 x 16 strip: the A
// fragments (rows) come from a double-buffered LDS tile filled with 16-byte
// copies of Ap; the B fragments (the wave's 16 columns) are read from Bt
// straight into registers, weighted by 2D/(D^2 + w^2) and split into NS parts
// there, once per element and frequency.  With four frequencies per workgroup
// (k_chi0_split8) eight waves share the tile: the B chunk goes through LDS as
// well, and each chunk of A and B is loaded once for the four frequencies.
// amax[mu] = max(amax[mu], largest |Re|, |Im| of B[k][mu] over 64 rows k) as
// float bits; one block per 64 rows of K
__global__ __launch_bounds__(256) void k_absmax_rows(const float2 *__restrict__ B, long long K, int N, unsigned *__restrict__ amax) {
  const long long k0 = (long long)blockIdx.x * 64;
  const long long k1 = k0 + 64 < K ? k0 + 64 : K;
  for (int mu = threadIdx.x; mu < N; mu += 256) {
    float m = 0.f;
    // 64 rows in blocks of 16 loads in flight (rows past K repeat row k0)
    for (long long kb = k0; kb < k1; kb += 16) {
      float2 v[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) v[t] = B[(kb + t < k1 ? kb + t : k0) * N + mu];
#pragma unroll
      for (int t = 0; t < 16; ++t) m = fmaxf(m, fmaxf(fabsf(v[t].x), fabsf(v[t].y)));
    }
    atomicMax(amax + mu, __float_as_uint(m));
  }
}

// 64 (k) x 32 (mu) tiles through LDS, 256 threads: the loads take 32
// consecutive mu of a row of B per 32 lanes; the stores, two k per thread,
// write 64 consecutive k of each mu row (512 bytes of Bt, 128 bytes of each
// part plane).  FP16 parts (H) and the FP32 copy Bt are taken of row mu times
// the power of two set by its largest magnitude amax[mu].  Columns k in
// [K, Kp) are written as zeros; Kp is a multiple of 32, so the last tile
// stops at Kp.
template <int NS, bool H>
__global__ __launch_bounds__(256) void k_chi0_presplit(const float2 *__restrict__ B, long long K, int N, long long Kp,
                                                       int Npad, const unsigned *__restrict__ amax, us16 *__restrict__ Ap,
                                                       float2 *__restrict__ Bt) {
  __shared__ float2 t[64][33];
  const long long k0 = (long long)blockIdx.x * 64;
  const int m0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int kk = ty + 8 * i;
    t[kk][tx] = ld_or(B, (k0 + kk) * N + m0 + tx, k0 + kk < K && m0 + tx < N, mkcf(0.f, 0.f));
  }
  __syncthreads();
  const long long k = k0 + 2 * tx;
  if (k >= Kp) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int mm = ty + 8 * j;
    float2 v0 = t[2 * tx][mm], v1 = t[2 * tx + 1][mm];
    if (H) {
      const float inv = m0 + mm < N ? inv_pow2_scale(__uint_as_float(amax[m0 + mm])) : 1.f;
      v0.x *= inv;
      v0.y *= inv;
      v1.x *= inv;
      v1.y *= inv;
    }
    const long long o = (long long)(m0 + mm) * Kp + k;   // even: 16-byte aligned in Bt, 4-byte in Ap
    *(float4 *)&Bt[o] = make_float4(v0.x, v0.y, v1.x, v1.y);
    us16 a0[NS], b0[NS], a1[NS], b1[NS];
    split_n<NS, H>(v0.x, a0);
    split_n<NS, H>(v0.y, b0);
    split_n<NS, H>(v1.x, a1);
    split_n<NS, H>(v1.y, b1);
#pragma unroll
    for (int p = 0; p < NS; ++p) {
      *(unsigned *)&Ap[(long long)(2 * p) * Npad * Kp + o] = (unsigned)a0[p] | ((unsigned)a1[p] << 16);
      *(unsigned *)&Ap[(long long)(2 * p + 1) * Npad * Kp + o] = (unsigned)b0[p] | ((unsigned)b1[p] << 16);
    }
  }
}

// Two frequencies per workgroup (NW = 2; four frequencies run in
// k_chi0_split8): the kernel is held to two waves per SIMD (232 registers),
// so one wave's weighting and splitting overlaps the other's products.
// FP16 parts (H): the weight of frequency w is taken times 2^-e_w with
// 2^e_w >= 1/w, which bounds |2D/(D^2 + w^2)| by 1, so the weighted, row-scaled
// B side stays below 2^15; the tile is scaled back by s_mu s_nu 2^e_w.
// A tile of the last tile row whose rows past N_aux fill whole 16-row blocks
// runs a copy of the chunk loop without those blocks' products (their
// partial-tile rows are never read).
template <int V> struct IntC { static constexpr int value = V; };
template <bool V> struct BoolC { static constexpr bool value = V; };

// One K chunk of a wave's 64 x 16 strip for NW frequencies: the wave's 16
// columns bcur (8 consecutive k per lane, FP32) are weighted by the rows wt0,
// wt0 + KCB, ... of the chunk's weight table, split into NS parts and
// multiplied with the A fragments of the NSI 16-row blocks in the LDS tile
// Asb: a conj(b), re = ar br + ai bi, im = ai br - ar bi, with the sign taken
// on the wave's own (weighted) side.
template <int NS, int NW, int NSI, int PAD, bool H>
__device__ __forceinline__ void chi0_chunk(const float2 (&bcur)[8], const float *wt0, const us16 (*Asb)[TILE][KCB + PAD],
                                           int col, int g, f4v (&re)[NW][4], f4v (&im)[NW][4]) {
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    float wt8[8];
    *(float4 *)&wt8[0] = *(const float4 *)&wt0[w * KCB + 8 * g];
    *(float4 *)&wt8[4] = *(const float4 *)&wt0[w * KCB + 8 * g + 4];
    u32x4 br[NS], bi[NS], nbi[NS];
    if constexpr (H && NS == 2) {
#pragma unroll
      for (int e = 0; e < 8; e += 2) {
        unsigned h, l;
        split2_h_pair(wt8[e], bcur[e].x, wt8[e + 1], bcur[e + 1].x, h, l);
        br[0][e / 2] = h;
        br[1][e / 2] = l;
        split2_h_pair(wt8[e], bcur[e].y, wt8[e + 1], bcur[e + 1].y, h, l);
        bi[0][e / 2] = h;
        bi[1][e / 2] = l;
      }
    } else {
      us16 brs[NS][8], bis[NS][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float wt = wt8[e];
        us16 pr_[NS], pi_[NS];
        split_n<NS, H>(wt * bcur[e].x, pr_);
        split_n<NS, H>(wt * bcur[e].y, pi_);
#pragma unroll
        for (int p = 0; p < NS; ++p) {
          brs[p][e] = pr_[p];
          bis[p][e] = pi_[p];
        }
      }
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        br[p] = *(const u32x4 *)brs[p];
        bi[p] = *(const u32x4 *)bis[p];
      }
    }
#pragma unroll
    for (int p = 0; p < NS; ++p) nbi[p] = bi[p] ^ 0x80008000u;
#pragma unroll
    for (int si = 0; si < NSI; ++si) {
#pragma unroll
      for (int p = 0; p < NS; ++p) {
        const u32x4 ar = *(const u32x4 *)&Asb[2 * p][16 * si + col][8 * g];
        const u32x4 ai = *(const u32x4 *)&Asb[2 * p + 1][16 * si + col][8 * g];
#pragma unroll
        for (int q = 0; q + p < NS; ++q) {
          re[w][si] = mfma_p<H>(ar, br[q], re[w][si]);
          re[w][si] = mfma_p<H>(ai, bi[q], re[w][si]);
          im[w][si] = mfma_p<H>(ai, br[q], im[w][si]);
          im[w][si] = mfma_p<H>(ar, nbi[q], im[w][si]);
        }
      }
    }
  }
}

// The wave's partial tiles (64 rows x its 16 columns cl, frequencies w0 ..
// w0 + NW - 1 of K split ks), scaled back by the row and column powers of two
// and the frequency's weight scale in the FP16 form.
template <int NW, bool H>
__device__ __forceinline__ void chi0_store(const f4v (&re)[NW][4], const f4v (&im)[NW][4], const float (&wsc)[NW], int w0,
                                           int n_freq, int ks, long long ntile, int tile, int mu0, int nu0, int cl, int N,
                                           int lane, const unsigned *__restrict__ amax, float2 *__restrict__ part) {
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w0 + w >= n_freq) continue;
    float2 *dst = part + (((long long)ks * n_freq + w0 + w) * ntile + tile) * (TILE * TILE);
    const float fcol = H ? pow2_scale(__uint_as_float(amax[nu0 + cl < N ? nu0 + cl : 0])) / wsc[w] : 1.f;
#pragma unroll
    for (int si = 0; si < 4; ++si) {
      if (16 * si >= N - mu0) break;
      const f4v r = re[w][si], i = im[w][si];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * si + Mfma<float>::row(lane, q);
        const float f = H ? fcol * pow2_scale(__uint_as_float(amax[mu0 + row < N ? mu0 + row : 0])) : 1.f;
        dst[row * TILE + cl] = mkcf(r[q] * f, i[q] * f);
      }
    }
  }
}

// The same for a swapped tile: the wave holds P[r][c] = sum_k a_r conj(w b_c)
// with r over 64 rows of column tile J (mu0 = J TILE) and c over the 16 rows
// of the last tile row (nu0); the tile (I, J) of the partial buffer is
// conj(P) transposed (the weight is real, so conj(P[r][c]) is the term of
// row nu0 + c and column mu0 + r).
template <int NW, bool H>
__device__ __forceinline__ void chi0_store_swapped(const f4v (&re)[NW][4], const f4v (&im)[NW][4], const float (&wsc)[NW],
                                                   int w0, int n_freq, int ks, long long ntile, int tile, int mu0,
                                                   int nu0, int N, int lane, const unsigned *__restrict__ amax,
                                                   float2 *__restrict__ part) {
  const int c = lane & 15;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (w0 + w >= n_freq) continue;
    float2 *dst = part + (((long long)ks * n_freq + w0 + w) * ntile + tile) * (TILE * TILE);
    const float fc = H ? pow2_scale(__uint_as_float(amax[nu0 + c < N ? nu0 + c : 0])) / wsc[w] : 1.f;
#pragma unroll
    for (int si = 0; si < 4; ++si) {
      if (16 * si >= N - mu0) break;
      const f4v r = re[w][si], i = im[w][si];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * si + Mfma<float>::row(lane, q);
        const float f = H ? fc * pow2_scale(__uint_as_float(amax[mu0 + row < N ? mu0 + row : 0])) : 1.f;
        dst[c * TILE + row] = mkcf(r[q] * f, -i[q] * f);
      }
    }
  }
}

// Work items of k_chi0_split8 over nt tile rows of N rows: (K split, tile,
// four frequencies) for every tile, except that a last tile row of at most 16
// rows is taken as (K split, column tile J, sixteen frequencies) with the roles
// of rows and columns swapped: such a work item weights and splits the 16 rows
// of the last tile row instead of the 64 columns of tile J.
__host__ __device__ inline bool split8_swap(int N, int nt) { return N - (nt - 1) * TILE <= 16; }
__host__ __device__ inline long long split8_items(int N, int nt, int n_freq, int nsplit) {
  const long long ntile = (long long)nt * (nt + 1) / 2;
  const bool sw = split8_swap(N, nt);
  return (long long)((n_freq + 3) / 4) * (sw ? ntile - nt : ntile) * nsplit +
         (sw ? (long long)((n_freq + 15) / 16) * nt * nsplit : 0);
}

template <int NS, int NW, int PAD, bool H>
__global__ __launch_bounds__(256, 2) void k_chi0_split(const us16 *__restrict__ Ap, const float2 *__restrict__ Bt,
                                                    const float *__restrict__ delta, const double *__restrict__ om2tab,
                                                    const double2 *__restrict__ cpltab, const float *__restrict__ wsctab, const int *__restrict__ wsel, const int *__restrict__ run, long long K,
                                                    long long Kp, int Npad, int n_freq, long long Ks, long long ntile,
                                                    const unsigned *__restrict__ amax, int N, float2 *__restrict__ part,
                                                    int nsplit) {
  if (run && *run == 0) return;
  __shared__ __attribute__((aligned(16))) us16 As[2][NS * 2][TILE][KCB + PAD];
  __shared__ __attribute__((aligned(16))) float wtab[2][NW][KCB];   // 2D/(D^2 + w^2) of the chunk
  // work item (K split s, tile, frequency group fg), fg fastest: each XCD
  // (workgroup id mod 8) takes a contiguous range, so the frequency groups
  // that read the same A and B slabs run back to back in one L2
  const int nfg = (n_freq + NW - 1) / NW;
  const long long total = (long long)nfg * ntile * nsplit, per = (total + 7) / 8;
  const long long wi = (long long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (wi >= total) return;
  const int fgi = (int)(wi % nfg);
  const int tile = (int)((wi / nfg) % ntile);
  const int ks = (int)(wi / ((long long)nfg * ntile));
  int I, J;
  tri_decode(tile, I, J);
  const int w0 = fgi * NW;
  const long long kb = (long long)ks * Ks;
  const long long ke = min(K, kb + Ks);
  const int mu0 = I * TILE, nu0 = J * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, g = lane >> 4;
  float om2[NW], wsc[NW], csv[NW];
  bool cim[NW];
  const bool cplx = cpltab != nullptr;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const bool in = w0 + w < n_freq;
    om2[w] = in ? (float)om2tab[wsel[w0 + w]] : 0.f;
    wsc[w] = (H && in) ? wsctab[wsel[w0 + w]] : 1.f;   // power of two, weight * wsc < 1
    const double2 cp = (cplx && in) ? cpltab[wsel[w0 + w]] : mkc(0.0, 0.0);
    csv[w] = (float)cp.x;
    cim[w] = cp.y != 0.0;
  }
  f4v re[NW][4], im[NW][4];
#pragma unroll
  for (int w = 0; w < NW; ++w)
#pragma unroll
    for (int si = 0; si < 4; ++si) re[w][si] = im[w][si] = Mfma<float>::zero();
  const int nch = (int)((ke - kb + KCB - 1) / KCB);
  if (nch <= 0) goto store;
  {
    // staging map of the A tile: thread -> (row, 8-k piece)
    const int arow = tid >> 2, ak = (tid & 3) * 8;
    const us16 *asrc = Ap + (long long)(mu0 + arow) * Kp + kb + ak;
    const long long pstride = (long long)Npad * Kp;
    const float2 *bsrc = Bt + (long long)(nu0 + 16 * wave + col) * Kp + kb + 8 * g;
    u32x4 apre[NS * 2];
    float2 bcur[8], bnext[8];
    // the weight table of a chunk is computed once per workgroup: thread t
    // < NW*KCB owns frequency t / KCB and row t % KCB
    const int tw = tid / KCB, tk = tid % KCB;
    // D of the chunk's row tk (the weights are formed from it after the
    // chunk's products, so no wait on the prefetches comes before them)
    auto dload = [&](long long k0) -> float {
      const long long k = k0 + tk;
      return (tw < NW && k < K) ? delta[k] : 1.f;
    };
    auto weight = [&](float dd) {
      const int w = tw < NW ? tw : 0;
      if (cplx) {
        const float a = dd * dd + om2[w];
        return 2.f * dd * (cim[w] ? csv[w] : a) / (a * a + csv[w] * csv[w]) * wsc[w];
      }
      return 2.f * dd / (dd * dd + om2[w]) * wsc[w];
    };
    float dnext = 1.f;
#pragma unroll
    for (int pr = 0; pr < NS * 2; ++pr) apre[pr] = *(const u32x4 *)(asrc + pr * pstride);
#pragma unroll
    for (int e = 0; e < 8; ++e) bcur[e] = bsrc[e];
    if (tw < NW) wtab[0][tw][tk] = weight(dload(kb));
#pragma unroll
    for (int pr = 0; pr < NS * 2; ++pr) *(u32x4 *)&As[0][pr][arow][ak] = apre[pr];
    // every load of the first chunk done: the loop then carries no pending
    // load into its first iteration, and its own waits cover only what it
    // issued itself
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    auto loop = [&](auto nsi_c) {
    constexpr int NSI = decltype(nsi_c)::value;
    for (int ch = 0; ch < nch; ++ch) {
      const int b = ch & 1;
      {
        // next chunk, clamped so that every iteration issues the same loads
        const long long off = (long long)min(ch + 1, nch - 1) * KCB;
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) apre[pr] = *(const u32x4 *)(asrc + pr * pstride + off);
#pragma unroll
        for (int e = 0; e < 8; ++e) bnext[e] = bsrc[off + e];
        dnext = dload(kb + off);
      }
      __builtin_amdgcn_sched_barrier(0);
      chi0_chunk<NS, NW, NSI, PAD, H>(bcur, &wtab[b][0][0], As[b], col, g, re, im);
      if (ch + 1 < nch) {
#pragma unroll
        for (int pr = 0; pr < NS * 2; ++pr) *(u32x4 *)&As[b ^ 1][pr][arow][ak] = apre[pr];
#pragma unroll
        for (int e = 0; e < 8; ++e) bcur[e] = bnext[e];
        if (tw < NW) wtab[b ^ 1][tw][tk] = weight(dnext);
      }
      __syncthreads();
    }
    };
    const int rem = N - mu0;
    if (rem > 2 * 16) loop(IntC<4>());
    else if (rem > 16) loop(IntC<2>());
    else loop(IntC<1>());
  }
store:
  chi0_store<NW, H>(re, im, wsc, w0, n_freq, ks, ntile, tile, mu0, nu0, 16 * wave + col, N, lane, amax, part);
}

// Eight waves per workgroup, four frequencies: waves w and w + 4 take the same
// 16 columns for frequency pairs 0 and 1, so the A and B chunks of a tile are
// loaded once (by all 512 threads, into double-buffered LDS) for four
// frequencies instead of two.  The B columns of a wave come from LDS in FP32
// and are weighted and split per frequency in registers as in k_chi0_split.
// When the last tile row holds at most 16 rows, its tiles run swapped (see
// split8_items): the eight waves take sixteen frequencies of the 16 weighted
// rows against the 64 unweighted rows of tile J, in place of four frequencies
// of 64 weighted columns against 16 or fewer rows.
template <int NS, int PAD, bool H, bool SWK>
__global__ __launch_bounds__(512) void k_chi0_split8(const us16 *__restrict__ Ap, const float2 *__restrict__ Bt,
                                                     const float *__restrict__ delta, const double *__restrict__ om2tab,
                                                     const double2 *__restrict__ cpltab, const float *__restrict__ wsctab,
                                                     const int *__restrict__ wsel, const int *__restrict__ run, long long K,
                                                     long long Kp, int Npad, int n_freq, long long Ks, long long ntile,
                                                     const unsigned *__restrict__ amax, int N, float2 *__restrict__ part,
                                                     int nsplit) {
  constexpr int NW = 2, NF = 4, NFS = 16;
  if (run && *run == 0) return;
  __shared__ __attribute__((aligned(16))) us16 As[2][NS * 2][TILE][KCB + PAD];
  __shared__ __attribute__((aligned(16))) float2 Bs[2][TILE][KCB + BBP];
  __shared__ __attribute__((aligned(16))) float wtab[2][SWK ? NFS : NF][KCB];
  // the plain work items first, then those of a swapped last tile row (SWK:
  // launched for the sizes that have one, split8_swap)
  const int nt = Npad / TILE;
  const bool sw = SWK;
  const long long nplain = sw ? ntile - nt : ntile;
  const int nfg = (n_freq + NF - 1) / NF, nfgs = (n_freq + NFS - 1) / NFS;
  const long long tplain = (long long)nfg * nplain * nsplit;
  const long long total = tplain + (sw ? (long long)nfgs * nt * nsplit : 0), per = (total + 7) / 8;
  const long long wi = (long long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (wi >= total) return;
  const bool swp = SWK && wi >= tplain;
  int fgi, tile, ks, I, J;
  if (!swp) {
    fgi = (int)(wi % nfg);
    tile = (int)((wi / nfg) % nplain);
    ks = (int)(wi / ((long long)nfg * nplain));
    tri_decode(tile, I, J);
  } else {
    const long long wj = wi - tplain;
    fgi = (int)(wj % nfgs);
    J = (int)((wj / nfgs) % nt);
    ks = (int)(wj / ((long long)nfgs * nt));
    I = nt - 1;
    tile = I * (I + 1) / 2 + J;
  }
  const long long kb = (long long)ks * Ks;
  const long long ke = min(K, kb + Ks);
  // rows mu0.. take the unweighted (A) side, columns nu0.. the weighted (B) side
  const int mu0 = (swp ? J : I) * TILE, nu0 = (swp ? I : J) * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, g = lane >> 4;
  // plain: waves w and w + 4 share 16 columns (two frequencies each);
  // swapped: all eight waves take the 16 columns, two frequencies each
  const int nf = swp ? NFS : NF;
  const int wcg = swp ? 0 : wave & 3, wf = swp ? wave : wave >> 2;
  const int w0 = fgi * nf + wf * NW;
  const bool cplx = cpltab != nullptr;
  float om2[NW], wsc[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const bool in = w0 + w < n_freq;
    om2[w] = in ? (float)om2tab[wsel[w0 + w]] : 0.f;
    wsc[w] = (H && in) ? wsctab[wsel[w0 + w]] : 1.f;
  }
  // the weight table: thread t < nf * KCB owns frequency fgi * nf + t / KCB and row t % KCB
  const int tw = tid / KCB, tk = tid % KCB;
  const bool wown = tw < nf && fgi * nf + tw < n_freq;
  const int fw_ = wown ? wsel[fgi * nf + tw] : 0;
  const float tom2 = wown ? (float)om2tab[fw_] : 0.f;
  const float twsc = (H && wown) ? wsctab[fw_] : 1.f;
  const double2 tcp = (cplx && wown) ? cpltab[fw_] : mkc(0.0, 0.0);
  const float tcsv = (float)tcp.x;
  const bool tcim = tcp.y != 0.0;
  auto weight = [&](float dd) {
    if (cplx) {
      const float a = dd * dd + tom2;
      return 2.f * dd * (tcim ? tcsv : a) / (a * a + tcsv * tcsv) * twsc;
    }
    return 2.f * dd / (dd * dd + tom2) * twsc;
  };
  // rows past K are zero in both operands: any finite weight serves
  auto dload = [&](long long k0) -> float { return delta[min(k0 + tk, K - 1)]; };
  f4v re[NW][4], im[NW][4];
#pragma unroll
  for (int w = 0; w < NW; ++w)
#pragma unroll
    for (int si = 0; si < 4; ++si) re[w][si] = im[w][si] = Mfma<float>::zero();
  const int nch = (int)((ke - kb + KCB - 1) / KCB);
  if (nch <= 0) goto store;
  {
    // A staging: plane parity ap, row arow, 8-k piece ak; B staging: column bc, 4-k piece bk
    const int ap = tid >> 8, arow = (tid >> 2) & 63, ak = (tid & 3) * 8;
    const int bc = tid >> 3, bk = (tid & 7) * 4;
    const bool bown = !swp || bc < 16;   // a swapped tile stages 16 columns (waves 0 and 1)
    const long long pstride = (long long)Npad * Kp;
    const us16 *asrc = Ap + (long long)ap * pstride + (long long)(mu0 + arow) * Kp + kb + ak;
    const float2 *bsrc = Bt + (long long)(nu0 + bc) * Kp + kb + bk;
    u32x4 apre[NS], bpre[2];
    float dnext = 1.f;
#pragma unroll
    for (int m = 0; m < NS; ++m) apre[m] = *(const u32x4 *)(asrc + 2 * m * pstride);
    if (bown) {
#pragma unroll
      for (int e = 0; e < 2; ++e) bpre[e] = *(const u32x4 *)(bsrc + 2 * e);
    }
    if (tw < nf) wtab[0][tw][tk] = weight(dload(kb));
#pragma unroll
    for (int m = 0; m < NS; ++m) *(u32x4 *)&As[0][ap + 2 * m][arow][ak] = apre[m];
    if (bown) {
#pragma unroll
      for (int e = 0; e < 2; ++e) *(u32x4 *)&Bs[0][bc][bk + 2 * e] = bpre[e];
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // the chunk loop, compiled apart for plain and swapped tiles
    auto loop = [&](auto nsi_c, auto swp_c) {
      constexpr int NSI = decltype(nsi_c)::value;
      constexpr bool SW = decltype(swp_c)::value;
      const bool bo = !SW || bc < 16;
      const bool wo = tw < (SW ? NFS : NF);
      for (int ch = 0; ch < nch; ++ch) {
        const int b = ch & 1;
        {
          const long long off = (long long)min(ch + 1, nch - 1) * KCB;
#pragma unroll
          for (int m = 0; m < NS; ++m) apre[m] = *(const u32x4 *)(asrc + 2 * m * pstride + off);
          if (bo) {
#pragma unroll
            for (int e = 0; e < 2; ++e) bpre[e] = *(const u32x4 *)(bsrc + off + 2 * e);
          }
          dnext = dload(kb + off);
        }
        __builtin_amdgcn_sched_barrier(0);
        // this wave's 16 columns of the chunk, 8 consecutive k per lane
        float2 bcur[8];
#pragma unroll
        for (int e = 0; e < 8; e += 2) *(u32x4 *)&bcur[e] = *(const u32x4 *)&Bs[b][16 * wcg + col][8 * g + e];
        chi0_chunk<NS, NW, NSI, PAD, H>(bcur, &wtab[b][wf * NW][0], As[b], col, g, re, im);
        {
#pragma unroll
          for (int m = 0; m < NS; ++m) *(u32x4 *)&As[b ^ 1][ap + 2 * m][arow][ak] = apre[m];
          if (bo) {
#pragma unroll
            for (int e = 0; e < 2; ++e) *(u32x4 *)&Bs[b ^ 1][bc][bk + 2 * e] = bpre[e];
          }
          if (wo) wtab[b ^ 1][tw][tk] = weight(dnext);
        }
        __syncthreads();
      }
    };
    const int rem = N - mu0;
    if constexpr (SWK) {
      if (swp) {
        // rows of a column tile J < nt - 1 fill it; the corner tile has at most 16
        if (rem > 16) loop(IntC<4>(), BoolC<true>());
        else loop(IntC<1>(), BoolC<true>());
        goto store;
      }
    }
    if (rem > 2 * 16) loop(IntC<4>(), BoolC<false>());
    else if (rem > 16) loop(IntC<2>(), BoolC<false>());
    else loop(IntC<1>(), BoolC<false>());
  }
store:
  if (SWK && swp) chi0_store_swapped<NW, H>(re, im, wsc, w0, n_freq, ks, ntile, tile, mu0, nu0, N, lane, amax, part);
  else chi0_store<NW, H>(re, im, wsc, w0, n_freq, ks, ntile, tile, mu0, nu0, 16 * wcg + col, N, lane, amax, part);
}

// chi[w][mu][nu] = scale * sum_s part[s][w][tile][..] (accumulate: added to
// chi's lower half as it stands); upper triangle by Hermitian symmetry.
template <typename T>
__global__ __launch_bounds__(256) void k_chi0_reduce(const typename c2t<T>::type *__restrict__ part, int S, int n_freq,
                                                     long long ntile, int N, double scale, const int *__restrict__ wsel,
                                                     const int *__restrict__ run, int accumulate,
                                                     typename c2t<T>::type *__restrict__ chi) {
  // one workgroup per (lower tile, frequency): the K-split partial tiles are
  // summed in FP64 along the tile's rows; the lower half of chi is written
  // along those rows, the mirrored upper half (conjugated) along the tile's
  // columns through an LDS transpose; the diagonal is made real
  using CT = typename c2t<T>::type;
  constexpr int E = TILE * TILE / 256;
  __shared__ CT tr[TILE][TILE + 1];
  if (run && *run == 0) return;
  const int t = blockIdx.x, w = blockIdx.y, tid = threadIdx.x;
  int I, J;
  tri_decode(t, I, J);
  const int mu0 = I * TILE, nu0 = J * TILE;
  double sr[E], si[E];
#pragma unroll
  for (int e = 0; e < E; ++e) sr[e] = si[e] = 0.0;
  const CT *src = part + ((long long)w * ntile + t) * (TILE * TILE);
  const long long sstride = (long long)n_freq * ntile * TILE * TILE;
  CT zero;
  zero.x = zero.y = 0;
  bool ok[E];
#pragma unroll
  for (int e = 0; e < E; ++e) ok[e] = mu0 + ((e * 256 + tid) >> 6) < N && nu0 + (tid & 63) < N;
  // every load of a step is issued before the first sum uses one
  auto step = [&](auto nsl_c, int s) {
    constexpr int NSL = decltype(nsl_c)::value;
    CT v[NSL][E];
#pragma unroll
    for (int l = 0; l < NSL; ++l)
#pragma unroll
      for (int e = 0; e < E; ++e) v[l][e] = ld_or(src + (s + l) * sstride, e * 256 + tid, ok[e], zero);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int l = 0; l < NSL; ++l)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        sr[e] += (double)v[l][e].x;
        si[e] += (double)v[l][e].y;
      }
  };
  int s = 0;
  for (; s + 2 <= S; s += 2) step(IntC<2>(), s);
  if (s < S) step(IntC<1>(), s);
  CT *dst = chi + (long long)wsel[w] * N * N;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int idx = e * 256 + tid, r = idx >> 6, cc = idx & 63;
    double2 z = mkc(scale * sr[e], scale * si[e]);
    const bool mine = mu0 + r < N && nu0 + cc < N && (I != J || cc <= r);
    if (accumulate && mine) {
      const CT o = dst[(long long)(mu0 + r) * N + nu0 + cc];
      z.x += (double)o.x;
      z.y += (double)o.y;
    }
    if (I == J && r == cc) z.y = 0.0;
    const CT v = to_c<T>(z);
    tr[r][cc] = v;
    if (mine) dst[(long long)(mu0 + r) * N + nu0 + cc] = v;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < E; ++e) {
    // output row nu0 + r2, column mu0 + c2 (upper half): conj of tile[c2][r2]
    const int idx = e * 256 + tid, r2 = idx >> 6, c2 = idx & 63;
    if (nu0 + r2 < N && mu0 + c2 < N && (I != J || c2 > r2)) {
      CT v = tr[c2][r2];
      v.y = -v.y;
      dst[(long long)(nu0 + r2) * N + mu0 + c2] = v;
    }
  }
}

// Number of K splits: enough workgroups to fill the device; in the split
// forms at most 2048 rows each.  The partial-tile buffer holds
// chi0_batch_splits of them; more are taken in batches (run_chi0_tab).
int chi0_plan_splits(const lrigw_ctx *c, int *splits) {
  const Dims &d = c->d;
  const long long K = lrigw_K(c);
  const int nt = (d.n_aux + TILE - 1) / TILE;
  const long long ntile = (long long)nt * (nt + 1) / 2;
  const int NW = c->chi_nw;
  const long long units = ntile * ((d.n_freq + NW - 1) / NW);
  long long S = (2048 + units - 1) / units;
  long long maxS = std::max<long long>(1, K / 512);
  S = std::min(S, maxS);
  if (ns_chi(c->precision) > 0) S = std::max(S, (K + 2047) / 2048);
  *splits = (int)std::max<long long>(1, S);
  return LRIGW_OK;
}

// Partial-tile buffer size: S splits of n_freq planes, at most 3 GiB (at
// least one split).
size_t chi0_part_bytes(const lrigw_ctx *c, int S) {
  const Dims &d = c->d;
  const int nt = (d.n_aux + TILE - 1) / TILE;
  const size_t per = (size_t)d.n_freq * ((size_t)nt * (nt + 1) / 2) * TILE * TILE * lrigw_csize(c);
  const size_t cap = std::max<size_t>(per, (size_t)3 << 30);
  return std::min<size_t>((size_t)S * per, cap / per * per);
}

static int check_gap(lrigw_ctx *c, const double *eig);

// every call reads the eigenvalues (new contents at the same address are
// checked too); the whole passes call it once and then open a GapScope
int chi0_check_gap(lrigw_ctx *c, const double *eig) { return check_gap(c, eig); }

static int check_gap(lrigw_ctx *c, const double *eig) {
  // insulator: every unoccupied level above every occupied level (D > 0)
  const Dims &d = c->d;
  std::vector<double> h((size_t)d.n_k * d.n_bands);
  LRIGW_HIP_TRY(hipMemcpyAsync(h.data(), eig, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  LRIGW_HIP_TRY(hipStreamSynchronize(c->stream));
  double vbm = -INFINITY, cbm = INFINITY;
  for (int k = 0; k < d.n_k; ++k)
    for (int n = 0; n < d.n_bands; ++n) {
      double e = h[(size_t)k * d.n_bands + n];
      if (!std::isfinite(e)) return LRIGW_ERR_ARG;
      if (n < d.n_occ) vbm = std::max(vbm, e);
      else cbm = std::min(cbm, e);
    }
  if (!(cbm > vbm)) return LRIGW_ERR_ARG;
  c->gap_min = cbm - vbm;
  double omax = -INFINITY, umax = -INFINITY, omin = INFINITY;
  for (int k = 0; k < d.n_k; ++k)
    for (int n = 0; n < d.n_bands; ++n) {
      const double e = h[(size_t)k * d.n_bands + n];
      if (n < d.n_occ) omin = std::min(omin, e), omax = std::max(omax, e);
      else umax = std::max(umax, e);
    }
  c->gap_max = umax - omin;
  return LRIGW_OK;
}

// chi at the frequencies wsel[0..n_sel) (device indices into the grid); when
// `run` is non-null the kernels do nothing unless *run != 0 (device flag).
int run_chi0_sel(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out, const int *wsel,
                 int n_sel, const int *run, bool real_axis) {
  const Dims &d = c->d;
  // per-plane tables: imaginary planes first, then the real-axis ones
  PlaneTab tab;
  tab.om2 = c->d_om2 + (real_axis ? d.n_freq : 0);
  tab.wsc = c->d_wsc + (real_axis ? d.n_freq : 0);
  tab.cpl = nullptr;
  return run_chi0_tab(c, iq, M, eig, apply_gamma, chi_out, wsel, n_sel, run, tab);
}

// chi at the planes wsel[0..n_sel) of the given per-plane tables
int run_chi0_tab(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out, const int *wsel,
                 int n_sel, const int *run, const PlaneTab &tab) {
  const Dims &d = c->d;
  const double *om2t = tab.om2;
  const float *wsct = tab.wsc;
  const double2 *cplt = tab.cpl;
  if (c->gap_trusted == 0) LRIGW_TRY(check_gap(c, eig));
  hipEvent_t ev_all;
  stage_begin(c, "chi0", &ev_all);
  LRIGW_TRY(launch_delta(c, iq, eig));
  const void *B = M;
  if (apply_gamma) {
    LRIGW_TRY(launch_gamma_modify(c, M));
    B = c->d_bhat;
  }
  const long long K = lrigw_K(c);
  const int nt = (d.n_aux + TILE - 1) / TILE;
  const long long ntile = (long long)nt * (nt + 1) / 2;
  const int S = c->chi_splits;
  const long long Ks = ((K + S - 1) / S + KCB - 1) / KCB * KCB;
  const double scale = -2.0 / d.n_k;
  // the partial-tile buffer holds Sb splits of these planes: the splits are
  // taken Sb at a time, each batch on rows k0.. of the operands (k0 a
  // multiple of KCB) and reduced into chi, the first batch writing it
  const size_t per = (size_t)n_sel * ntile * TILE * TILE * lrigw_csize(c);
  const int Sb = (int)std::max<size_t>(1, std::min<size_t>((size_t)S, c->part_bytes / per));
  if ((size_t)Sb * per > c->part_bytes) return LRIGW_ERR_ARG;   // more planes than the buffer was sized for
  const int NW = c->chi_nw;
  const bool split = c->precision != LRIGW_FP64 && c->precision != LRIGW_FP32;
  const long long Kp = (K + KCB - 1) / KCB * KCB;
  const int Npad = nt * TILE;
  hipEvent_t ev;
  if (split) {
    stage_begin(c, "chi0_split", &ev);
    const float2 *Bf = (const float2 *)B;
    us16 *Apd = (us16 *)c->d_ap;
    float2 *Btd = (float2 *)c->d_bt;
    dim3 pg((unsigned)((Kp + 63) / 64), (unsigned)(Npad / 32));
    const int NS = ns_chi(c->precision);
    const bool H = split_h(c->precision);
    if (H) {
      LRIGW_TRY(zero_fill(c->stream, c->d_amax, (size_t)Npad * sizeof(unsigned)));
      hipLaunchKernelGGL(k_absmax_rows, dim3((unsigned)((K + 63) / 64)), dim3(256), 0, c->stream, Bf, K, d.n_aux, c->d_amax);
      hipLaunchKernelGGL((k_chi0_presplit<2, true>), pg, dim3(256), 0, c->stream, Bf, K, d.n_aux, Kp, Npad, c->d_amax, Apd,
                         Btd);
    } else if (NS == 2) {
      hipLaunchKernelGGL((k_chi0_presplit<2, false>), pg, dim3(256), 0, c->stream, Bf, K, d.n_aux, Kp, Npad, nullptr, Apd,
                         Btd);
    } else {
      hipLaunchKernelGGL((k_chi0_presplit<3, false>), pg, dim3(256), 0, c->stream, Bf, K, d.n_aux, Kp, Npad, nullptr, Apd,
                         Btd);
    }
    stage_end(c, "chi0_split", ev);
  }
  for (int s0 = 0; s0 < S; s0 += Sb) {
    const long long k0 = (long long)s0 * Ks;
    if (k0 >= K) break;
    const int sb = std::min(Sb, S - s0);
    const long long Kb = K - k0;   // rows from k0 on; split ks of the batch covers [ks Ks, (ks+1) Ks)
    stage_begin(c, "chi0_mfma", &ev);
    if (c->precision == LRIGW_FP64) {
      dim3 grid((unsigned)ntile, (n_sel + NW - 1) / NW, sb);
      const double2 *Bb = (const double2 *)B + k0 * d.n_aux;
      const double *Db = (const double *)c->d_delta + k0;
#define CHI0_ARGS om2t, cplt, wsel, run, Kb, d.n_aux, n_sel, Ks, ntile
      if (NW == 2)
        hipLaunchKernelGGL((k_chi0_mfma<double, 2>), grid, dim3(256), 0, c->stream, Bb, Db, CHI0_ARGS, (double2 *)c->d_part);
      else
        hipLaunchKernelGGL((k_chi0_mfma<double, 1>), grid, dim3(256), 0, c->stream, Bb, Db, CHI0_ARGS, (double2 *)c->d_part);
    } else if (c->precision == LRIGW_FP32) {
      dim3 grid((unsigned)ntile, (n_sel + NW - 1) / NW, sb);
      const float2 *Bb = (const float2 *)B + k0 * d.n_aux;
      const float *Db = (const float *)c->d_delta + k0;
      float2 *Pf = (float2 *)c->d_part;
      if (NW == 4) hipLaunchKernelGGL((k_chi0_mfma<float, 4>), grid, dim3(256), 0, c->stream, Bb, Db, CHI0_ARGS, Pf);
      else hipLaunchKernelGGL((k_chi0_mfma<float, 2>), grid, dim3(256), 0, c->stream, Bb, Db, CHI0_ARGS, Pf);
#undef CHI0_ARGS
    } else {
      const us16 *Apb = (const us16 *)c->d_ap + k0;
      const float2 *Btb = (const float2 *)c->d_bt + k0;
      const float *Db = (const float *)c->d_delta + k0;
      float2 *Pf = (float2 *)c->d_part;
      const bool p16 = c->chi_pad == 16;
      const int NS = ns_chi(c->precision);
      const bool H = split_h(c->precision);
      // 1D over (K split, tile, frequency group), split over the XCDs
      const long long sitems = NW == 4 ? split8_items(d.n_aux, nt, n_sel, sb) : (long long)((n_sel + NW - 1) / NW) * ntile * sb;
      const dim3 sgrid((unsigned)(8 * ((sitems + 7) / 8)));
#define BF16_ARGS Apb, Btb, Db, om2t, cplt, wsct, wsel, run, Kb, Kp, Npad, n_sel, Ks, ntile, c->d_amax, d.n_aux, Pf, sb
      const bool swk = split8_swap(d.n_aux, nt);
#define SPLIT_LAUNCH(NS_, H_)                                                                                            \
  do {                                                                                                                 \
    if (NW == 4 && swk && p16)                                                                                         \
      hipLaunchKernelGGL((k_chi0_split8<NS_, 16, H_, true>), sgrid, dim3(512), 0, c->stream, BF16_ARGS);              \
    else if (NW == 4 && swk)                                                                                           \
      hipLaunchKernelGGL((k_chi0_split8<NS_, 8, H_, true>), sgrid, dim3(512), 0, c->stream, BF16_ARGS);               \
    else if (NW == 4 && p16)                                                                                           \
      hipLaunchKernelGGL((k_chi0_split8<NS_, 16, H_, false>), sgrid, dim3(512), 0, c->stream, BF16_ARGS);             \
    else if (NW == 4)                                                                                                  \
      hipLaunchKernelGGL((k_chi0_split8<NS_, 8, H_, false>), sgrid, dim3(512), 0, c->stream, BF16_ARGS);              \
    else if (p16) hipLaunchKernelGGL((k_chi0_split<NS_, 2, 16, H_>), sgrid, dim3(256), 0, c->stream, BF16_ARGS);      \
    else hipLaunchKernelGGL((k_chi0_split<NS_, 2, 8, H_>), sgrid, dim3(256), 0, c->stream, BF16_ARGS);                \
  } while (0)
      if (H) SPLIT_LAUNCH(2, true);
      else if (NS == 2) SPLIT_LAUNCH(2, false);
      else SPLIT_LAUNCH(3, false);
#undef SPLIT_LAUNCH
#undef BF16_ARGS
    }
    stage_end(c, "chi0_mfma", ev);
    LRIGW_TRY(lrigw_launch_check("chi0_mfma"));
    dim3 rgrid((unsigned)ntile, n_sel);
    const int acc = s0 > 0;
    if (c->precision == LRIGW_FP64)
      hipLaunchKernelGGL(k_chi0_reduce<double>, rgrid, dim3(256), 0, c->stream, (const double2 *)c->d_part, sb, n_sel, ntile,
                         d.n_aux, scale, wsel, run, acc, (double2 *)chi_out);
    else
      hipLaunchKernelGGL(k_chi0_reduce<float>, rgrid, dim3(256), 0, c->stream, (const float2 *)c->d_part, sb, n_sel, ntile,
                         d.n_aux, scale, wsel, run, acc, (float2 *)chi_out);
  }
  LRIGW_TRY(lrigw_launch_check("chi0_reduce"));
  stage_end(c, "chi0", ev_all);
  return LRIGW_OK;
}

int run_chi0(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out) {
  return run_chi0_sel(c, iq, M, eig, apply_gamma, chi_out, c->d_wall, c->d.n_freq, nullptr);
}
