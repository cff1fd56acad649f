// Exchange self-energy: the bare-Coulomb term of Eq. GW_selfe_element
// (W_0 = V + W^c).  V does not depend on the frequency, and with the
// equal-time convergence factor of the exchange term the frequency integral
// keeps the occupied bands only:
//   Sigma^x_n(k) = -1/N_q sum_q sum_{m occ} sum_{mu nu} x^mu V_{mu nu}(q) conj(x^nu),
// x^mu = C^mu_{nm}(k,k-q) (the pairing of the self-energy equation: the second
// coefficient C^nu_{mn}(k-q,k) is conj(x^nu)), V(0) the truncated Coulomb
// matrix as in the screening (Sec. III B).  The sum is real (V Hermitian) and
// equals Re sum_mu conj(x^mu) Z^mu with Z = V^* x, i.e. Z = X V^H for the rows
// of X.  Per q, in FP64 (V is FP64): Z on the batched FP64 MFMA GEMM (a row of
// X is one pair (k, n, m), its N_aux coefficients contiguous), then one wave
// per (k, n) sums Re(conj(X) Z) over m and mu in a fixed order.
#include <algorithm>

#include "lrigw_internal.h"
#include "tiles.h"

template <typename CIN>
__global__ void k_sx_widen(const CIN *__restrict__ in, double2 *__restrict__ out, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) out[i] = to_z(in[i]);
}

// sx[k][n] += -(1/N_q) sum_{m < n_occ} sum_mu Re(conj(X[p][mu]) Z[p][mu]),
// p = (k n_qp + n) n_occ + m; one wave per (k, n)
__global__ __launch_bounds__(256) void k_sx_reduce(const double2 *__restrict__ X, const double2 *__restrict__ Z,
                                                   int n_kqp, int n_occ, int N, double scale, double *__restrict__ sx) {
  const int kn = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (kn >= n_kqp) return;
  const long long base = (long long)kn * n_occ * N;
  const long long len = (long long)n_occ * N;
  double s = 0.0;
  for (long long e = lane; e < len; e += 64) {
    const double2 a = X[base + e], z = Z[base + e];
    s += a.x * z.x + a.y * z.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) sx[kn] += scale * s;
}

static int sx_buffers(lrigw_ctx *c) {
  const Dims &d = c->d;
  const size_t pairs = (size_t)d.n_k * d.n_qp * d.n_occ * d.n_aux;
  if (!c->d_sxz) LRIGW_HIP_TRY(hipMalloc(&c->d_sxz, pairs * sizeof(double2)));
  if (c->precision != LRIGW_FP64 && !c->d_sxa) LRIGW_HIP_TRY(hipMalloc(&c->d_sxa, pairs * sizeof(double2)));
  return LRIGW_OK;
}

int run_sigma_x(lrigw_ctx *c, int iq, const void *xo, const void *V, double *sigma_x) {
  (void)iq;
  const Dims &d = c->d;
  const int n = d.n_aux;
  const long long rows = (long long)d.n_k * d.n_qp * d.n_occ;
  if (rows == 0) return LRIGW_OK;
  LRIGW_TRY(sx_buffers(c));
  hipStream_t s = c->stream;
  const double2 *X;
  if (c->precision == LRIGW_FP64) {
    X = (const double2 *)xo;
  } else {
    const long long tot = rows * n;
    hipLaunchKernelGGL(k_sx_widen<float2>, dim3((unsigned)std::min<long long>((tot + 255) / 256, 16384)), dim3(256), 0, s,
                       (const float2 *)xo, (double2 *)c->d_sxa, tot);
    X = (const double2 *)c->d_sxa;
  }
  // Z = X V^H: Z[p][mu] = sum_nu conj(V[mu][nu]) X[p][nu]
  ZGemm g;
  g.m = (int)rows; g.n = n; g.k = n;
  g.opa = OP_N; g.A = X; g.lda = n; g.sa = 0;
  g.opb = OP_C; g.B = (const double2 *)V; g.ldb = n; g.sb = 0;
  g.C = (double2 *)c->d_sxz; g.ldc = n; g.sc = 0;
  g.alpha = mkc(1.0, 0.0); g.beta = mkc(0.0, 0.0);
  g.batch = 1; g.lower_only = 0;
  LRIGW_TRY(zgemm(s, g));
  const int n_kqp = d.n_k * d.n_qp;
  hipLaunchKernelGGL(k_sx_reduce, dim3((unsigned)((n_kqp + 3) / 4)), dim3(256), 0, s, X, (const double2 *)c->d_sxz, n_kqp,
                     d.n_occ, n, -1.0 / (double)d.n_k, sigma_x);
  return lrigw_launch_check("sigma_x");
}
