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

#define LP (TILE + 1)   // padded LDS row (complex elements)

template <typename T>
__global__ __launch_bounds__(256) void k_sigma_mfma(const typename c2t<T>::type *__restrict__ x, const typename c2t<T>::type *__restrict__ Wall,
                                                    long long Ccols, int N, T *__restrict__ Xall) {
  typedef typename c2t<T>::type C;
  typedef Mfma<T> MF;
  typedef typename MF::acc ACC;
  __shared__ C Wt[TILE][LP];   // Wt[nu][mu] = W[mu][nu] (block I, J)
  __shared__ C Ut[TILE][LP];   // Ut[nu][c]  = conj(x[c][nu])
  __shared__ T red[2][TILE];

  const C *W = Wall + (long long)blockIdx.y * N * N;
  T *Xout = Xall + (long long)blockIdx.y * Ccols;
  const long long c0 = (long long)blockIdx.x * TILE;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, col = lane & 15;
  const int nt = (N + TILE - 1) / TILE;
  T psum[2] = {(T)0, (T)0};

  for (int I = 0; I < nt; ++I) {
    const int mu0 = I * TILE;
    ACC zr[2][2], zi[2][2];
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) {
        zr[si][sj] = MF::zero();
        zi[si][sj] = MF::zero();
      }
    for (int J = 0; J <= I; ++J) {
      const int nu0 = J * TILE;
      const bool diag = (J == I);
      __syncthreads();
      // W block rows mu (64) x cols nu (64), 16 consecutive nu per thread group
#pragma unroll 4
      for (int t = 0; t < (TILE * TILE) / 256; ++t) {
        int e = tid + 256 * t;
        int m = e / TILE, kk = e % TILE;
        int mu = mu0 + m, nu = nu0 + kk;
        C w;
        w.x = w.y = (T)0;
        if (mu < N && nu < N && (!diag || nu < mu)) w = W[(long long)mu * N + nu];
        Wt[kk][m] = w;
        long long cc = c0 + m;
        C u;
        u.x = u.y = (T)0;
        if (cc < Ccols && nu < N) u = cconj(x[cc * N + nu]);
        Ut[kk][m] = u;
      }
      __syncthreads();
#pragma unroll 4
      for (int ks = 0; ks < TILE / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        C wv[2], uv[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          wv[s] = Wt[kk][32 * wr + 16 * s + col];
          uv[s] = Ut[kk][32 * wc + 16 * s + col];
        }
#pragma unroll
        for (int si = 0; si < 2; ++si)
#pragma unroll
          for (int sj = 0; sj < 2; ++sj) {
            // Z += W u: re = Wr ur - Wi ui, im = Wr ui + Wi ur
            zr[si][sj] = MF::mac(wv[si].x, uv[sj].x, zr[si][sj]);
            zr[si][sj] = MF::mac(-wv[si].y, uv[sj].y, zr[si][sj]);
            zi[si][sj] = MF::mac(wv[si].x, uv[sj].y, zi[si][sj]);
            zi[si][sj] = MF::mac(wv[si].y, uv[sj].x, zi[si][sj]);
          }
      }
    }
    // epilogue of row block I: Ut holds conj(x) of block I (last J == I)
#pragma unroll
    for (int si = 0; si < 2; ++si)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int ml = 32 * wr + 16 * si + MF::row(lane, q);
          const int cl = 32 * wc + 16 * sj + col;
          const int mu = mu0 + ml;
          if (mu < N) {
            C u = Ut[ml][cl];                       // conj(x_mu)
            T xr = u.x, xi = -u.y;                  // x_mu
            T wdd = (T)W[(long long)mu * N + mu].x;
            // 2 Re(x Z) + Re W_mumu |x|^2
            psum[sj] += (T)2 * (xr * zr[si][sj][q] - xi * zi[si][sj][q]) + wdd * (xr * xr + xi * xi);
          }
        }
  }
  // lanes l, l^16, l^32, l^48 hold the same column
#pragma unroll
  for (int sj = 0; sj < 2; ++sj) {
    T v = psum[sj];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    psum[sj] = v;
  }
  __syncthreads();
  if (lane < 16) {
#pragma unroll
    for (int sj = 0; sj < 2; ++sj) red[wr][32 * wc + 16 * sj + lane] = psum[sj];
  }
  __syncthreads();
  if (tid < TILE) {
    long long cc = c0 + tid;
    if (cc < Ccols) Xout[cc] = red[0][tid] + red[1][tid];
  }
}

// sigma[k][n][i] += scale * sum_m sum_j g_j X[j][k][n][m] a/(a^2 + w_j^2),  a = i w_i + mu - e_m(k-q)
template <typename T>
__global__ void k_sigma_freq(const T *__restrict__ X, const double *__restrict__ eig, const int *__restrict__ kmq, int iq,
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
    const T *xp = X + ((long long)k * n_qp + n) * n_bands + m;
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
  else
    hipLaunchKernelGGL(k_sigma_mfma<float>, grid, dim3(256), 0, c->stream, (const float2 *)x, (const float2 *)Wc, Ccols,
                       d.n_aux, (float *)c->d_X);
  stage_end(c, "sigma_mfma", ev);
  LRIGW_TRY(lrigw_launch_check("sigma_mfma"));
  long long tot = (long long)d.n_k * d.n_qp * d.n_freq;
  dim3 g2((unsigned)((tot + 127) / 128));
  const double scale = -1.0 / (M_PI * d.n_k);
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_sigma_freq<double>, g2, dim3(128), 0, c->stream, (const double *)c->d_X, eig, c->d_kmq, iq, d.n_k,
                       d.n_qp, d.n_bands, d.n_freq, c->d_omega, c->d_weight, d.mu, scale, (double2 *)sigma_acc);
  else
    hipLaunchKernelGGL(k_sigma_freq<float>, g2, dim3(128), 0, c->stream, (const float *)c->d_X, eig, c->d_kmq, iq, d.n_k,
                       d.n_qp, d.n_bands, d.n_freq, c->d_omega, c->d_weight, d.mu, scale, (double2 *)sigma_acc);
  LRIGW_TRY(lrigw_launch_check("sigma_freq"));
  stage_end(c, "sigma_c", ev_all);
  return LRIGW_OK;
}
