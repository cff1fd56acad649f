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

template <typename T>
__global__ __launch_bounds__(256) void k_chi0_mfma(const typename c2t<T>::type *__restrict__ B, const T *__restrict__ delta,
                                                   const double *__restrict__ omega, long long K, int N, int n_freq, long long Ks,
                                                   long long ntile, typename c2t<T>::type *__restrict__ part) {
  typedef typename c2t<T>::type C;
  typedef Mfma<T> MF;
  typedef typename MF::acc ACC;
  const int NW = Chi0Cfg<T>::NW;
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

  T om2[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    double o = (w0 + w < n_freq) ? omega[w0 + w] : 0.0;
    om2[w] = (T)(o * o);
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
        const T wt = (T)2 * d / (d * d + om2[w]);
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

// chi[w][mu][nu] = scale * sum_s part[s][w][tile][..]; upper triangle by Hermitian symmetry.
template <typename T>
__global__ void k_chi0_reduce(const typename c2t<T>::type *__restrict__ part, int S, int n_freq, long long ntile, int N,
                              double scale, typename c2t<T>::type *__restrict__ chi) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int w = blockIdx.y;
  if (idx >= (long long)N * N) return;
  int mu = (int)(idx / N), nu = (int)(idx % N);
  bool up = nu > mu;
  int a = up ? nu : mu, b = up ? mu : nu;
  int I = a / TILE, J = b / TILE;
  long long t = (long long)I * (I + 1) / 2 + J;
  long long off = (long long)(a % TILE) * TILE + (b % TILE);
  double sr = 0.0, si = 0.0;
  for (int s = 0; s < S; ++s) {
    auto v = part[(((long long)s * n_freq + w) * ntile + t) * (TILE * TILE) + off];
    sr += (double)v.x;
    si += (double)v.y;
  }
  double2 z = mkc(scale * sr, scale * si);
  if (up) z.y = -z.y;
  if (mu == nu) z.y = 0.0;
  chi[((long long)w * N + mu) * N + nu] = to_c<T>(z);
}

// Number of K splits: enough workgroups to fill the device, partial buffer <= 2 GiB.
int chi0_plan_splits(const lrigw_ctx *c, int *splits) {
  const Dims &d = c->d;
  const long long K = lrigw_K(c);
  const int nt = (d.n_aux + TILE - 1) / TILE;
  const long long ntile = (long long)nt * (nt + 1) / 2;
  const int NW = c->precision == LRIGW_FP64 ? Chi0Cfg<double>::NW : Chi0Cfg<float>::NW;
  const long long units = ntile * ((d.n_freq + NW - 1) / NW);
  long long S = (2048 + units - 1) / units;
  long long maxS = std::max<long long>(1, K / 512);
  S = std::min(S, maxS);
  const size_t cs = lrigw_csize(c);
  const size_t per = (size_t)d.n_freq * ntile * TILE * TILE * cs;
  while (S > 1 && (size_t)S * per > (size_t)2 << 30) --S;
  *splits = (int)std::max<long long>(1, S);
  return LRIGW_OK;
}

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
  return LRIGW_OK;
}

int run_chi0(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out) {
  const Dims &d = c->d;
  if (eig != c->checked_eig) {
    LRIGW_TRY(check_gap(c, eig));
    c->checked_eig = eig;
  }
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
  const long long Ks = ((K + S - 1) / S + KC - 1) / KC * KC;
  const double scale = -2.0 / d.n_k;
  hipEvent_t ev;
  stage_begin(c, "chi0_mfma", &ev);
  if (c->precision == LRIGW_FP64) {
    const int NW = Chi0Cfg<double>::NW;
    dim3 grid((unsigned)ntile, (d.n_freq + NW - 1) / NW, S);
    hipLaunchKernelGGL(k_chi0_mfma<double>, grid, dim3(256), 0, c->stream, (const double2 *)B, (const double *)c->d_delta,
                       c->d_omega, K, d.n_aux, d.n_freq, Ks, ntile, (double2 *)c->d_part);
  } else {
    const int NW = Chi0Cfg<float>::NW;
    dim3 grid((unsigned)ntile, (d.n_freq + NW - 1) / NW, S);
    hipLaunchKernelGGL(k_chi0_mfma<float>, grid, dim3(256), 0, c->stream, (const float2 *)B, (const float *)c->d_delta,
                       c->d_omega, K, d.n_aux, d.n_freq, Ks, ntile, (float2 *)c->d_part);
  }
  stage_end(c, "chi0_mfma", ev);
  LRIGW_TRY(lrigw_launch_check("chi0_mfma"));
  dim3 rgrid((unsigned)(((long long)d.n_aux * d.n_aux + 255) / 256), d.n_freq);
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_chi0_reduce<double>, rgrid, dim3(256), 0, c->stream, (const double2 *)c->d_part, S, d.n_freq, ntile,
                       d.n_aux, scale, (double2 *)chi_out);
  else
    hipLaunchKernelGGL(k_chi0_reduce<float>, rgrid, dim3(256), 0, c->stream, (const float2 *)c->d_part, S, d.n_freq, ntile,
                       d.n_aux, scale, (float2 *)chi_out);
  LRIGW_TRY(lrigw_launch_check("chi0_reduce"));
  stage_end(c, "chi0", ev_all);
  return LRIGW_OK;
}
