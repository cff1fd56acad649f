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
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

#define SKC 16          // nu rows staged per step
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
                                                    long long Ccols, int N, double *__restrict__ Xall) {
  typedef typename c2t<T>::type C;
  typedef Mfma<T> MF;
  typedef typename MF::acc ACC;
  __shared__ C Ws[2][SKC][SLP];   // Ws[b][nu][mu] = W[mu][nu] for the current group
  __shared__ C Us[2][SKC][SLP];   // Us[b][nu][c]  = conj(x[c][nu])
  __shared__ double red[4][TILE];

  const C *W = Wall + (long long)blockIdx.y * N * N;
  double *Xout = Xall + (long long)blockIdx.y * Ccols;
  const long long c0 = (long long)blockIdx.x * TILE;
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

// Split-BF16 form: W^c and conj(x) are split into NS BF16 parts when staged in
// LDS, products of parts p + q < NS are accumulated by the 16x16x32 BF16 MFMA
// in FP32.  Same work decomposition as k_sigma_mfma, nu chunks of 32.
#define SKB 32
#define SBP 8

template <int NS>
__device__ inline void splitn_s(float v, __bf16 *p) {
  float r = v;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    p[i] = (__bf16)r;
    r -= (float)p[i];
  }
}

template <int NS>
__global__ __launch_bounds__(256) void k_sigma_bf16(const float2 *__restrict__ x, const float2 *__restrict__ Wall, long long Ccols,
                                                    int N, double *__restrict__ Xall) {
  __shared__ __bf16 Wr[NS][TILE][SKB + SBP], Wi[NS][TILE][SKB + SBP];   // [part][mu][nu]
  __shared__ __bf16 Ur[NS][TILE][SKB + SBP], Ui[NS][TILE][SKB + SBP];   // [part][c][nu] of conj(x)
  __shared__ double red[4][TILE];
  const float2 *W = Wall + (long long)blockIdx.y * N * N;
  double *Xout = Xall + (long long)blockIdx.y * Ccols;
  const long long c0 = (long long)blockIdx.x * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, col = lane & 15, g = lane >> 4;
  const int ngroups = (N + TILE - 1) / TILE;
  const int base = N - ngroups * TILE;
  double psum[4] = {0.0, 0.0, 0.0, 0.0};
  const int lrow = tid >> 5, lk = tid & 31;     // 32 consecutive threads read 32 nu of one row; rows lrow + 8 t

  for (int I = 0; I < ngroups; ++I) {
    const int mu0 = base + I * TILE;
    const int nch = (mu0 + TILE - 2 >= 0) ? (mu0 + TILE - 2) / SKB + 1 : 1;
    const int r0 = mu0 + 16 * wave;
    const bool active = (r0 + 15 >= 0);
    const int kcw = active ? ((r0 + 14 >= 0) ? (r0 + 14) / SKB + 1 : 1) : 0;
    f4v zr[4], zi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) zr[j] = zi[j] = Mfma<float>::zero();
    float2 wreg[8], ureg[8];
    auto fetch = [&](int ch) {
      const int nu = ch * SKB + lk;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int m = lrow + 8 * t;
        const int mu = mu0 + m;
        float2 w = mkcf(0.f, 0.f);
        if (mu >= 0 && mu < N && nu < mu) w = W[(long long)mu * N + nu];
        wreg[t] = w;
        const long long cc = c0 + m;
        float2 u = mkcf(0.f, 0.f);
        if (cc < Ccols && nu < N) u = cconj(x[cc * N + nu]);
        ureg[t] = u;
      }
    };
    auto stash = [&]() {
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int m = lrow + 8 * t;
        __bf16 a[NS], b[NS], c[NS], d[NS];
        splitn_s<NS>(wreg[t].x, a);
        splitn_s<NS>(wreg[t].y, b);
        splitn_s<NS>(ureg[t].x, c);
        splitn_s<NS>(ureg[t].y, d);
#pragma unroll
        for (int p = 0; p < NS; ++p) {
          Wr[p][m][lk] = a[p];
          Wi[p][m][lk] = b[p];
          Ur[p][m][lk] = c[p];
          Ui[p][m][lk] = d[p];
        }
      }
    };
    fetch(0);
    for (int ch = 0; ch < nch; ++ch) {
      __syncthreads();
      stash();
      __syncthreads();
      if (ch + 1 < nch) fetch(ch + 1);
      if (ch < kcw) {
        bf16x8 ar[NS], ai[NS], nai[NS];
#pragma unroll
        for (int p = 0; p < NS; ++p) {
          ar[p] = *(const bf16x8 *)&Wr[p][16 * wave + col][8 * g];
          ai[p] = *(const bf16x8 *)&Wi[p][16 * wave + col][8 * g];
          nai[p] = -ai[p];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          bf16x8 ur[NS], ui[NS];
#pragma unroll
          for (int p = 0; p < NS; ++p) {
            ur[p] = *(const bf16x8 *)&Ur[p][16 * j + col][8 * g];
            ui[p] = *(const bf16x8 *)&Ui[p][16 * j + col][8 * g];
          }
          // Z += W u: re = Wr ur - Wi ui, im = Wr ui + Wi ur
#pragma unroll
          for (int p = 0; p < NS; ++p)
#pragma unroll
            for (int q = 0; q + p < NS; ++q) {
              zr[j] = mfma_bf16(ar[p], ur[q], zr[j]);
              zr[j] = mfma_bf16(nai[p], ui[q], zr[j]);
              zi[j] = mfma_bf16(ar[p], ui[q], zi[j]);
              zi[j] = mfma_bf16(ai[p], ur[q], zi[j]);
            }
        }
      }
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long long cc = c0 + 16 * j + col;
        if (cc >= Ccols) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int mu = r0 + Mfma<float>::row(lane, q);
          if (mu < 0 || mu >= N) continue;
          const float2 xv = x[cc * N + mu];
          const double wdd = (double)W[(long long)mu * N + mu].x;
          const double xr = (double)xv.x, xi = (double)xv.y;
          psum[j] += 2.0 * (xr * (double)zr[j][q] - xi * (double)zi[j][q]) + wdd * (xr * xr + xi * xi);
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    double v = psum[j];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    psum[j] = v;
  }
  __syncthreads();
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

// sigma[k][n][i] += scale * sum_m sum_j g_j X[j][k][n][m] a/(a^2 + w_j^2),  a = i w_i + mu - e_m(k-q)
__global__ void k_sigma_freq(const double *__restrict__ X, const double *__restrict__ eig, const int *__restrict__ kmq, int iq,
                             int nk, int n_qp, int n_bands, int n_freq, const double *__restrict__ omega,
                             const double *__restrict__ weight, double mu, double scale, double2 *__restrict__ sigma) {
  long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = (long long)nk * n_qp * n_freq;
  if (idx >= tot) return;
  const int i = (int)(idx % n_freq);
  const int n = (int)((idx / n_freq) % n_qp);
  const int k = (int)(idx / ((long long)n_freq * n_qp));
  const int k2 = kmq[k * nk + iq];
  const double wi = omega[i];
  const long long cstride = (long long)nk * n_qp * n_bands;
  double sr = 0.0, si = 0.0;
  for (int m = 0; m < n_bands; ++m) {
    const double ar = mu - eig[(long long)k2 * n_bands + m];
    const double ai = wi;
    const double *xp = X + ((long long)k * n_qp + n) * n_bands + m;
    for (int j = 0; j < n_freq; ++j) {
      const double wj = omega[j];
      const double dr = ar * ar - ai * ai + wj * wj, di = 2.0 * ar * ai;
      const double inv = 1.0 / (dr * dr + di * di);
      const double kr = (ar * dr + ai * di) * inv, ki = (ai * dr - ar * di) * inv;
      const double gx = weight[j] * (double)xp[(long long)j * cstride];
      sr += gx * kr;
      si += gx * ki;
    }
  }
  const long long o = ((long long)k * n_qp + n) * n_freq + i;
  double2 s = sigma[o];
  s.x += scale * sr;
  s.y += scale * si;
  sigma[o] = s;
}

int run_sigma_c(lrigw_ctx *c, int iq, const void *x, const void *Wc, const double *eig, void *sigma_acc) {
  const Dims &d = c->d;
  const long long Ccols = (long long)d.n_k * d.n_qp * d.n_bands;
  hipEvent_t ev_all, ev;
  stage_begin(c, "sigma_c", &ev_all);
  stage_begin(c, "sigma_mfma", &ev);
  dim3 grid((unsigned)((Ccols + TILE - 1) / TILE), d.n_freq);
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_sigma_mfma<double>, grid, dim3(256), 0, c->stream, (const double2 *)x, (const double2 *)Wc, Ccols,
                       d.n_aux, (double *)c->d_X);
  else if (c->precision == LRIGW_FP32)
    hipLaunchKernelGGL(k_sigma_mfma<float>, grid, dim3(256), 0, c->stream, (const float2 *)x, (const float2 *)Wc, Ccols,
                       d.n_aux, (double *)c->d_X);
  else if (c->precision == LRIGW_SPLIT_BF16)
    hipLaunchKernelGGL(k_sigma_bf16<2>, grid, dim3(256), 0, c->stream, (const float2 *)x, (const float2 *)Wc, Ccols,
                       d.n_aux, (double *)c->d_X);
  else
    hipLaunchKernelGGL(k_sigma_bf16<3>, grid, dim3(256), 0, c->stream, (const float2 *)x, (const float2 *)Wc, Ccols,
                       d.n_aux, (double *)c->d_X);
  stage_end(c, "sigma_mfma", ev);
  LRIGW_TRY(lrigw_launch_check("sigma_mfma"));
  long long tot = (long long)d.n_k * d.n_qp * d.n_freq;
  dim3 g2((unsigned)((tot + 127) / 128));
  const double scale = -1.0 / (M_PI * d.n_k);
  hipLaunchKernelGGL(k_sigma_freq, g2, dim3(128), 0, c->stream, (const double *)c->d_X, eig, c->d_kmq, iq, d.n_k, d.n_qp,
                     d.n_bands, d.n_freq, c->d_omega, c->d_weight, d.mu, scale, (double2 *)sigma_acc);
  LRIGW_TRY(lrigw_launch_check("sigma_freq"));
  stage_end(c, "sigma_c", ev_all);
  return LRIGW_OK;
}
