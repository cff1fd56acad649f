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
#include <mutex>

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

// The fit on caller-provided workspace: Vz [batch][n][n] and Yz [batch][n][nrhs]
// complex128, Dinv [batch][zdinv_stride(n)] complex128, dinfo 4 ints.
static int lri_fit_core(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T,
                        double scale, double *C, int *info, double2 *Vz, double2 *Yz, double2 *Dinv, int *dinfo) {
  hipStream_t s = c->stream;
  const long long nn = (long long)n * n, nr = (long long)n * nrhs;
  int rc = LRIGW_OK;
  const unsigned gv = (unsigned)std::min<long long>((batch * nn + 255) / 256, 16384);
  const unsigned gt = (unsigned)std::min<long long>((batch * nr + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fit_to_z, dim3(gv), dim3(256), 0, s, V, Vz, batch * nn);
  hipLaunchKernelGGL(k_fit_to_z, dim3(gt), dim3(256), 0, s, T, Yz, batch * nr);
  LRIGW_TRY(lrigw_launch_check("lri_fit_in"));
  // V = L L^H, then Y <- L^{-H} L^{-1} T
  if ((rc = zpotrf_batched(s, Vz, n, n, nn, batch, Dinv, dinfo)) < 0 ||
      (rc = ztrsm_left_lower(s, Vz, n, nn, Dinv, Yz, nrhs, nr, n, nrhs, batch)) < 0 ||
      (rc = ztrsm_left_upper_conj(s, Vz, n, nn, Dinv, Yz, nrhs, nr, n, nrhs, batch)) < 0)
    return rc;
  const unsigned gc = (unsigned)std::min<long long>(((long long)batch * n_keep * nrhs + 255) / 256, 16384);
  hipLaunchKernelGGL(k_fit_take, dim3(gc), dim3(256), 0, s, Yz, n, n_keep, nrhs, (long long)batch, scale, C);
  LRIGW_TRY(lrigw_launch_check("lri_fit_out"));
  int h = INT_MAX;
  if (hipMemcpyAsync(&h, dinfo, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return LRIGW_ERR_HIP;
  if (info) *info = (h == INT_MAX) ? -1 : h;
  return (h == INT_MAX) ? LRIGW_OK : LRIGW_ERR_NOT_HPD;
}

int run_lri_fit(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T, double scale,
                double *C, int *info) {
  const long long nn = (long long)n * n, nr = (long long)n * nrhs;
  double2 *Vz = nullptr, *Yz = nullptr, *Dinv = nullptr;
  int *dinfo = nullptr;
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
  const int rc = lri_fit_core(c, batch, n, n_keep, nrhs, V, T, scale, C, info, Vz, Yz, Dinv, dinfo);
  if (rc < 0) (void)hipStreamSynchronize(c->stream);   // queued work may still use the workspace
  cleanup();
  return rc;
}

// ---------------------------------------------------------------- allocation-free variant
// The workspace of lrigw_lri_fit_noalloc lives in this fixed device array.
// Host code never passes `scratch` itself to a kernel: in host code the name
// is a host-side stand-in, not a device address.  Its device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and kept in fit_scratch_ptr[]; every use goes through that pointer.  Each
// device holds its own copy until the process ends; calls that overlap on one
// device share it and race.
static __device__ __align__(256) unsigned char scratch[LRIGW_FIT_SCRATCH_BYTES];

static std::mutex fit_scratch_mu;
static void *fit_scratch_ptr[LRIGW_MAX_DEVICES] = {};

int fit_scratch_prepare(int dev) {
  if (dev < 0 || dev >= LRIGW_MAX_DEVICES) return LRIGW_ERR_ARG;
  std::lock_guard<std::mutex> lock(fit_scratch_mu);
  if (fit_scratch_ptr[dev]) return LRIGW_OK;
  int cur = -1;
  LRIGW_HIP_TRY(hipGetDevice(&cur));
  if (cur != dev) LRIGW_HIP_TRY(hipSetDevice(dev));
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess) return lrigw_hip_error(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
  if (!p) return LRIGW_ERR_HIP;
  fit_scratch_ptr[dev] = p;
  return LRIGW_OK;
}

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

// bytes of scratch the fit of this shape needs
size_t fit_scratch_bytes(int batch, int n, int nrhs) {
  const size_t nn = (size_t)n * n, nr = (size_t)n * nrhs;
  return up256(4 * sizeof(int)) + up256((size_t)batch * nn * sizeof(double2)) +
         up256((size_t)batch * nr * sizeof(double2)) + up256((size_t)batch * zdinv_stride(n) * sizeof(double2));
}

int run_lri_fit_noalloc(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T,
                        double scale, double *C, int *info) {
  const double need = (double)fit_scratch_bytes(batch, n, nrhs);
  if (need > (double)LRIGW_FIT_SCRATCH_BYTES) return LRIGW_ERR_ARG;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(fit_scratch_mu);
    if (c->device >= 0 && c->device < LRIGW_MAX_DEVICES) base = fit_scratch_ptr[c->device];
  }
  if (!base) {   // first call on a device whose context did not prepare it
    LRIGW_TRY(fit_scratch_prepare(c->device));
    std::lock_guard<std::mutex> lock(fit_scratch_mu);
    base = fit_scratch_ptr[c->device];
  }
  const size_t nn = (size_t)n * n, nr = (size_t)n * nrhs;
  char *p = (char *)base;
  int *dinfo = (int *)p;
  p += up256(4 * sizeof(int));
  double2 *Vz = (double2 *)p;
  p += up256((size_t)batch * nn * sizeof(double2));
  double2 *Yz = (double2 *)p;
  p += up256((size_t)batch * nr * sizeof(double2));
  double2 *Dinv = (double2 *)p;
  // every element of the workspace is written before it is read (the inputs
  // are copied in, the Cholesky status word is set by its own init kernel and
  // the diagonal-block inverses by the factorisation), so nothing needs
  // clearing between calls
  return lri_fit_core(c, batch, n, n_keep, nrhs, V, T, scale, C, info, Vz, Yz, Dinv, dinfo);
}
