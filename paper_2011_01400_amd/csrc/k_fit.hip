// Two-centre LRI coefficients (Eq. two_center_coeff_determination): for a
// batch of atom pairs of one shape, the first n_keep rows of V^{-1} T, with V
// the Coulomb matrix of the pair's auxiliary functions and T the integrals
// (ij|nu), one column per orbital product.  V is real symmetric positive
// definite; the solve reuses the batched FP64 Cholesky (64x64 diagonal blocks
// factored and inverted in LDS, panels and trailing updates on the FP64 MFMA
// GEMM) and the two triangular solves, on the real matrices carried as
// complex with zero imaginary part.
#include <algorithm>
#include <climits>

#include "lrigw_internal.h"
#include "tiles.h"

__global__ void k_fit_to_z(const double *__restrict__ in, double2 *__restrict__ out, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) out[i] = mkc(in[i], 0.0);
}

// C[b][r][c] = scale * Re Y[b][r][c] for r < n_keep
__global__ void k_fit_take(const double2 *__restrict__ Y, int n, int n_keep, int nrhs, long long batch, double scale,
                           double *__restrict__ C) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)n_keep * nrhs, tot = per * batch;
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; i < tot; i += st) {
    const long long b = i / per, e = i % per;
    C[i] = scale * Y[b * n * (long long)nrhs + e].x;
  }
}

int run_lri_fit(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T, double scale,
                double *C, int *info) {
  hipStream_t s = c->stream;
  const long long nn = (long long)n * n, nr = (long long)n * nrhs;
  double2 *Vz = nullptr, *Yz = nullptr, *Dinv = nullptr;
  int *dinfo = nullptr;
  int rc = LRIGW_OK;
  auto cleanup = [&]() {
    if (Vz) (void)hipFree(Vz);
    if (Yz) (void)hipFree(Yz);
    if (Dinv) (void)hipFree(Dinv);
    if (dinfo) (void)hipFree(dinfo);
  };
  if (hipMalloc(&Vz, (size_t)batch * nn * sizeof(double2)) != hipSuccess ||
      hipMalloc(&Yz, (size_t)batch * nr * sizeof(double2)) != hipSuccess ||
      hipMalloc(&Dinv, (size_t)batch * zdinv_stride(n) * sizeof(double2)) != hipSuccess ||
      hipMalloc(&dinfo, 4 * sizeof(int)) != hipSuccess) {
    cleanup();
    return LRIGW_ERR_OOM;
  }
  const unsigned gv = (unsigned)std::min<long long>((batch * nn + 255) / 256, 16384);
  const unsigned gt = (unsigned)std::min<long long>((batch * nr + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fit_to_z, dim3(gv), dim3(256), 0, s, V, Vz, batch * nn);
  hipLaunchKernelGGL(k_fit_to_z, dim3(gt), dim3(256), 0, s, T, Yz, batch * nr);
  if ((rc = lrigw_launch_check("lri_fit_in")) < 0) { cleanup(); return rc; }
  // V = L L^H, then Y <- L^{-H} L^{-1} T
  if ((rc = zpotrf_batched(s, Vz, n, n, nn, batch, Dinv, dinfo)) < 0 ||
      (rc = ztrsm_left_lower(s, Vz, n, nn, Dinv, Yz, nrhs, nr, n, nrhs, batch)) < 0 ||
      (rc = ztrsm_left_upper_conj(s, Vz, n, nn, Dinv, Yz, nrhs, nr, n, nrhs, batch)) < 0) {
    cleanup();
    return rc;
  }
  const unsigned gc = (unsigned)std::min<long long>(((long long)batch * n_keep * nrhs + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fit_take, dim3(gc), dim3(256), 0, s, Yz, n, n_keep, nrhs, (long long)batch, scale, C);
  if ((rc = lrigw_launch_check("lri_fit_out")) < 0) { cleanup(); return rc; }
  int h = INT_MAX;
  if (hipMemcpyAsync(&h, dinfo, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return LRIGW_ERR_HIP;
  }
  cleanup();
  if (info) *info = (h == INT_MAX) ? -1 : h;
  return (h == INT_MAX) ? LRIGW_OK : LRIGW_ERR_NOT_HPD;
}
