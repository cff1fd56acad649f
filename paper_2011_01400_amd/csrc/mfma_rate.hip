// Sustained dense FP16 matrix-core rate of the device, the reference against
// which the MFMA kernels' fractions of the published peak are read.
//
// Every wave of 1024 workgroups x 256 threads (four waves per SIMD on 256
// CUs) runs eight independent v_mfma_f32_16x16x32_f16 chains for a fixed
// number of iterations; the launch time (HIP events) gives the rate.  Each
// workgroup also records the shader-clock counter (s_memtime) and the 100 MHz
// reference counter (s_memrealtime) around its loop, whose ratio is the mean
// shader clock while it ran.  The operands are all zeros, then uniform in
// [-1, 1): the power drawn by the matrix cores depends on the operand bits,
// and with random operands the clock drops below its peak.
//
// Output: one JSON line {"instruction", "zeros": {pflops, mhz}, "random":
// {pflops, mhz}} with the median over the repetitions after the first.
// Exit status 0 on success, 1 on a HIP error (message on stdout).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

#define CK(x)                                                                        \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) {                                                          \
      printf("{\"error\": \"%s at line %d\"}\n", hipGetErrorString(e_), __LINE__); \
      return 1;                                                                      \
    }                                                                                \
  } while (0)

// two workgroups per CU fit in registers; the eight accumulators start from
// different values so that no two chains are the same computation
__global__ __launch_bounds__(256, 2) void k_mfma_rate(const h8 *__restrict__ a, const h8 *__restrict__ b,
                                                      float *__restrict__ out, long long *__restrict__ clk, int iters) {
  const int tid = blockIdx.x * 256 + threadIdx.x;
  const h8 x = a[tid], y = b[tid];
  const float z = (float)(tid & 1);
  f4 c0 = {z, 0.f, 0.f, 0.f}, c1 = {1.f, z, 0.f, 0.f}, c2 = {2.f, 0.f, z, 0.f}, c3 = {3.f, 0.f, 0.f, z};
  f4 c4 = {4.f, z, z, 0.f}, c5 = {5.f, 0.f, z, z}, c6 = {6.f, z, 0.f, z}, c7 = {7.f, z, z, z};
  const long long t0 = __builtin_readcyclecounter();
  const long long r0 = __builtin_amdgcn_s_memrealtime();
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c3, 0, 0, 0);
    c4 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c4, 0, 0, 0);
    c5 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c5, 0, 0, 0);
    c6 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c6, 0, 0, 0);
    c7 = __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c7, 0, 0, 0);
  }
  const long long t1 = __builtin_readcyclecounter();
  const long long r1 = __builtin_amdgcn_s_memrealtime();
  const f4 s = c0 + c1 + c2 + c3 + c4 + c5 + c6 + c7;
  out[tid] = s[0] + s[1] + s[2] + s[3];
  if (threadIdx.x == 0) {
    clk[2 * blockIdx.x] = t1 - t0;
    clk[2 * blockIdx.x + 1] = r1 - r0;
  }
}

int main() {
  const int nblk = 1024, nthr = nblk * 256, iters = 100000, reps = 4;
  h8 *a, *b;
  float *out;
  long long *clk;
  CK(hipMalloc(&a, sizeof(h8) * nthr));
  CK(hipMalloc(&b, sizeof(h8) * nthr));
  CK(hipMalloc(&out, sizeof(float) * nthr));
  CK(hipMalloc(&clk, sizeof(long long) * 2 * nblk));
  hipEvent_t e0, e1;
  CK(hipEventCreate(&e0));
  CK(hipEventCreate(&e1));
  std::vector<h8> ha(nthr), hb(nthr);
  std::vector<long long> hc(2 * nblk);
  std::mt19937 gen(7);
  std::uniform_real_distribution<float> uni(-1.f, 1.f);
  const double flops = (double)nthr / 64 * iters * 8 * (2.0 * 16 * 16 * 32);
  double pf[2], mhz[2];
  for (int mode = 0; mode < 2; ++mode) {
    for (int i = 0; i < nthr; ++i)
      for (int e = 0; e < 8; ++e) {
        ha[i][e] = (_Float16)(mode ? uni(gen) : 0.f);
        hb[i][e] = (_Float16)(mode ? uni(gen) : 0.f);
      }
    CK(hipMemcpy(a, ha.data(), sizeof(h8) * nthr, hipMemcpyHostToDevice));
    CK(hipMemcpy(b, hb.data(), sizeof(h8) * nthr, hipMemcpyHostToDevice));
    std::vector<double> r_pf, r_mhz;
    for (int rep = 0; rep < reps; ++rep) {
      CK(hipEventRecord(e0, 0));
      hipLaunchKernelGGL(k_mfma_rate, dim3(nblk), dim3(256), 0, 0, a, b, out, clk, iters);
      CK(hipGetLastError());
      CK(hipEventRecord(e1, 0));
      CK(hipEventSynchronize(e1));
      float ms = 0.f;
      CK(hipEventElapsedTime(&ms, e0, e1));
      CK(hipMemcpy(hc.data(), clk, sizeof(long long) * 2 * nblk, hipMemcpyDeviceToHost));
      double cy = 0.0, rt = 0.0;
      for (int i = 0; i < nblk; ++i) {
        cy += (double)hc[2 * i];
        rt += (double)hc[2 * i + 1];
      }
      if (rep == 0) continue;   // the first launch ramps the clock
      r_pf.push_back(flops / (ms * 1e-3) / 1e15);
      r_mhz.push_back(cy / rt * 100.0);
    }
    std::sort(r_pf.begin(), r_pf.end());
    std::sort(r_mhz.begin(), r_mhz.end());
    pf[mode] = r_pf[r_pf.size() / 2];
    mhz[mode] = r_mhz[r_mhz.size() / 2];
  }
  printf("{\"instruction\": \"v_mfma_f32_16x16x32_f16\", \"zeros\": {\"pflops\": %.4f, \"mhz\": %.0f}, "
         "\"random\": {\"pflops\": %.4f, \"mhz\": %.0f}}\n",
         pf[0], mhz[0], pf[1], mhz[1]);
  CK(hipFree(a));
  CK(hipFree(b));
  CK(hipFree(out));
  CK(hipFree(clk));
  return 0;
}
