// MO triple coefficients (Eqs. AO_triple_split2 and AO_MO_transform) and the
// q = 0 head/wing preparation (Sec. III B).
#include <algorithm>
#include <cmath>

#include "lrigw_internal.h"
#include "tiles.h"

// M[k][r][c][mu] = sum_{a on atom(mu)} conj(c_{a,r0+r}(k)) H[k2][a][c0+c][mu] + conj(H[k][a][r0+r][mu]) c_{a,c0+c}(k2)
// k2 = kmap[k][iq].  One thread per (mu, 4 columns c); NR >= nr row accumulators
// per column, so every H[k][a][r][mu] loaded serves BM_CPT columns
// (BM_CPT * NR <= 32 keeps the accumulators in registers).  Workgroup ->
// (mu block, column block, k): each XCD (workgroup id mod 8) takes a
// contiguous range of the work items, column block fastest, so the column
// blocks of one (mu block, k) share the row panel H[k][.][r][mu] in that XCD's
// L2 instead of fetching it once per column block.
template <typename T, int NR, int BM_CPT>
__global__ __launch_bounds__(256) void k_build_M(const typename c2t<T>::type *__restrict__ H, const double2 *__restrict__ evec,
                                                 int n_bands, int n_b, int n_aux, int nb_max, const int *__restrict__ aux_atom,
                                                 const int *__restrict__ basis_off, const int *__restrict__ kmap, int iq,
                                                 int nk, int r0, int nr, int c0, int nc, int rr0, int nr_tot,
                                                 typename c2t<T>::type *__restrict__ M) {
  typedef typename c2t<T>::type C;
  const int nmb = (n_aux + 63) / 64, ncb = (nc + 4 * BM_CPT - 1) / (4 * BM_CPT);
  const long long total = (long long)nmb * ncb * nk, per = (total + 7) / 8;
  const long long w = (long long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (w >= total) return;
  const int yb = (int)(w % ncb), xb = (int)((w / ncb) % nmb), k = (int)(w / ((long long)ncb * nmb));
  const int mu = xb * 64 + (threadIdx.x & 63);
  const int cb = (yb * 4 + (threadIdx.x >> 6)) * BM_CPT;   // first column of this thread
  if (mu >= n_aux || cb >= nc) return;
  const int A = aux_atom[mu];
  const int bo = basis_off[A];
  const int nbA = basis_off[A + 1] - bo;
  const int k2 = kmap[k * nk + iq];
  const int ncol = min(BM_CPT, nc - cb);
  C acc[BM_CPT][NR];
#pragma unroll
  for (int t = 0; t < BM_CPT; ++t)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[t][r].x = acc[t][r].y = (T)0;
  // padded columns (t >= ncol) and rows (r >= nr) repeat a valid one: their
  // accumulators are never stored, and with no guard around them the loads of
  // a basis function are all in flight together
  for (int a = 0; a < nbA; ++a) {
    C h2[BM_CPT], e2[BM_CPT], h1[NR], e1[NR];
    const C *h2row = H + (((long long)k2 * nb_max + a) * n_bands + c0 + cb) * n_aux + mu;
    const double2 *e2row = evec + ((long long)k2 * n_b + bo + a) * n_bands + c0 + cb;
    const C *h1row = H + (((long long)k * nb_max + a) * n_bands + r0) * n_aux + mu;
    const double2 *e1row = evec + ((long long)k * n_b + bo + a) * n_bands + r0;
    double2 e2d[BM_CPT], e1d[NR];
#pragma unroll
    for (int t = 0; t < BM_CPT; ++t) {
      const int tt = min(t, ncol - 1);
      h2[t] = h2row[(long long)tt * n_aux];
      e2d[t] = e2row[tt];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int rr = min(r, nr - 1);
      h1[r] = h1row[(long long)rr * n_aux];
      e1d[r] = e1row[rr];
    }
#pragma unroll
    for (int t = 0; t < BM_CPT; ++t) {
      e2[t].x = (T)e2d[t].x;
      e2[t].y = (T)e2d[t].y;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      e1[r].x = (T)e1d[r].x;
      e1[r].y = (T)e1d[r].y;
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int t = 0; t < BM_CPT; ++t) acc[t][r] = cadd(acc[t][r], cadd(ccmul(e1[r], h2[t]), ccmul(h1[r], e2[t])));
  }
#pragma unroll
  for (int t = 0; t < BM_CPT; ++t)
    if (t < ncol)
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nr) M[(((long long)k * nr_tot + rr0 + r) * nc + cb + t) * n_aux + mu] = acc[t][r];
}

// The same sums with the eigenvector rows the workgroup needs held in LDS in
// the compute type (E1[b][r] = c_{b,r0+r}(k), E2[b][t] = c_{b,c0+colb+t}(k2)
// for every basis function b): a wave then loads only H, and the H values of
// basis function a + 1 are fetched into a second register set while those of
// a are used.  Lanes of one wave may belong to different atoms (loop lengths
// differ per lane; no barrier follows the staging one).
template <typename T, int NR, int CPT>
__global__ __launch_bounds__(256) void k_build_M_lds(const typename c2t<T>::type *__restrict__ H, const double2 *__restrict__ evec,
                                                     int n_bands, int n_b, int n_aux, int nb_max, const int *__restrict__ aux_atom,
                                                     const int *__restrict__ basis_off, const int *__restrict__ kmap, int iq,
                                                     int nk, int r0, int nr, int c0, int nc, int rr0, int nr_tot,
                                                     typename c2t<T>::type *__restrict__ M) {
  typedef typename c2t<T>::type C;
  // thread <-> one entry of the flattened (column group of CPT columns, mu)
  // space of one k point, mu fastest, 256 entries per workgroup: a wave may
  // straddle two column groups, and no wave is left with a few lanes of a
  // last mu block.  Each XCD (workgroup id mod 8) takes a contiguous range of
  // workgroups, so those of one k share its row panel in one L2.
  const int ngr = (nc + CPT - 1) / CPT;
  const long long per_k = (long long)ngr * n_aux;
  const int wgk = (int)((per_k + 255) / 256);
  const long long total = (long long)wgk * nk, per = (total + 7) / 8;
  const long long w = (long long)(blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (w >= total) return;
  const int k = (int)(w / wgk);
  const long long f0 = (w % wgk) * 256;
  const int g0 = (int)(f0 / n_aux);                        // first column group of the workgroup
  const int g1 = (int)min((long long)ngr - 1, (f0 + 255) / n_aux);
  const int BC = (g1 - g0 + 1) * CPT;                      // columns staged
  extern __shared__ __attribute__((aligned(16))) unsigned char bm_smem[];
  C *E1s = (C *)bm_smem;        // [n_b][NR]
  C *E2s = E1s + n_b * NR;      // [n_b][BC]
  const int k2 = kmap[k * nk + iq];
  const int tid = threadIdx.x;
  const int colb = g0 * CPT;
  for (int e = tid; e < n_b * NR; e += 256) {
    const int b = e / NR, r = min(e % NR, nr - 1);
    const double2 v = evec[((long long)k * n_b + b) * n_bands + r0 + r];
    E1s[e].x = (T)v.x;
    E1s[e].y = (T)v.y;
  }
  for (int e = tid; e < n_b * BC; e += 256) {
    const int b = e / BC, t = min(colb + e % BC, nc - 1);
    const double2 v = evec[((long long)k2 * n_b + b) * n_bands + c0 + t];
    E2s[e].x = (T)v.x;
    E2s[e].y = (T)v.y;
  }
  __syncthreads();
  const long long f = f0 + tid;
  if (f >= per_k) return;
  const int gi = (int)(f / n_aux), mu = (int)(f - (long long)gi * n_aux);
  const int cb = gi * CPT;          // first column of this thread
  const int lcol = cb - colb;       // its offset among the staged columns
  const int A = aux_atom[mu];
  const int bo = basis_off[A];
  const int nbA = basis_off[A + 1] - bo;
  const int ncol = min(CPT, nc - cb);
  // offsets inside one k point's H block (nb_max * n_bands * n_aux elements)
  // in 32 bits
  const int astr = n_bands * n_aux;
  const C *h2base = H + ((long long)k2 * nb_max * n_bands + c0 + cb) * n_aux + mu;
  const C *h1base = H + ((long long)k * nb_max * n_bands + r0) * n_aux + mu;
  C acc[CPT][NR];
#pragma unroll
  for (int t = 0; t < CPT; ++t)
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[t][r].x = acc[t][r].y = (T)0;
  // padded columns (t >= ncol) and rows (r >= nr) repeat a valid one; their
  // accumulators are never stored
  auto ld = [&](C (&x2)[CPT], C (&x1)[NR], int a) {
#pragma unroll
    for (int t = 0; t < CPT; ++t) x2[t] = h2base[a * astr + min(t, ncol - 1) * n_aux];
#pragma unroll
    for (int r = 0; r < NR; ++r) x1[r] = h1base[a * astr + min(r, nr - 1) * n_aux];
  };
  auto step = [&](const C (&x2)[CPT], const C (&x1)[NR], int a) {
    const C *e1 = E1s + (bo + a) * NR;
    const C *e2 = E2s + (bo + a) * BC + lcol;
    C ev1[NR], ev2[CPT];
#pragma unroll
    for (int r = 0; r < NR; ++r) ev1[r] = e1[r];
#pragma unroll
    for (int t = 0; t < CPT; ++t) ev2[t] = e2[t];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int t = 0; t < CPT; ++t) acc[t][r] = cadd(acc[t][r], cadd(ccmul(ev1[r], x2[t]), ccmul(x1[r], ev2[t])));
  };
  if (nbA > 0) {
    // an odd first basis function is taken alone, so the paired loop has no
    // branch; the scheduling barriers keep each prefetch ahead of the step it
    // overlaps
    C h2[CPT], h1[NR], n2[CPT], n1[NR];
    int a = nbA & 1;
    if (a) ld(n2, n1, 0);
    ld(h2, h1, a);
    if (a) step(n2, n1, 0);
    for (; a < nbA; a += 2) {
      ld(n2, n1, a + 1);
      __builtin_amdgcn_sched_barrier(0);
      step(h2, h1, a);
      ld(h2, h1, min(a + 2, nbA - 1));
      __builtin_amdgcn_sched_barrier(0);
      step(n2, n1, a + 1);
    }
  }
#pragma unroll
  for (int t = 0; t < CPT; ++t)
    if (t < ncol)
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (r < nr) M[(((long long)k * nr_tot + rr0 + r) * nc + cb + t) * n_aux + mu] = acc[t][r];
}

// LDS of the staged eigenvector rows (bytes); above this the direct-load form runs
#define BM_LDS_MAX (64 * 1024)

template <typename T>
static void launch_build(lrigw_ctx *c, int iq, int r0, int nr, int c0, int nc, const int *kmap, const void *H,
                         const void *evec, void *M) {
  typedef typename c2t<T>::type C;
  const Dims &d = c->d;
  const long long nmb = (d.n_aux + 63) / 64;
#define BM_GRID(CPT) dim3((unsigned)(8 * ((nmb * ((nc + 4 * CPT - 1) / (4 * CPT)) * d.n_k + 7) / 8)))
  // flattened form: 256 (column group, mu) entries per workgroup, staging the
  // eigenvector columns of at most 256 / n_aux + 2 column groups
#define BML_WGK(CPT) ((((long long)(nc + CPT - 1) / CPT) * d.n_aux + 255) / 256)
#define BML_GRID(CPT) dim3((unsigned)(8 * ((BML_WGK(CPT) * d.n_k + 7) / 8)))
#define BML_GROUPS(CPT) std::min<long long>((nc + CPT - 1) / CPT, 256 / d.n_aux + 2)
#define BM_ARGS(NRV) (const C *)H, (const double2 *)evec, d.n_bands, d.n_b, d.n_aux, d.nb_max, c->d_aux_atom, c->d_basis_off, \
                     kmap, iq, d.n_k, r0 + rb, nrl, c0, nc, rb, nr, (C *)M
#define BM(NRV, CPT) hipLaunchKernelGGL((k_build_M<T, NRV, CPT>), BM_GRID(CPT), dim3(256), 0, c->stream, BM_ARGS(NRV))
#define BML(NRV, CPT)                                                                                               \
  hipLaunchKernelGGL((k_build_M_lds<T, NRV, CPT>), BML_GRID(CPT), dim3(256),                                        \
                     (size_t)d.n_b * (NRV + BML_GROUPS(CPT) * CPT) * sizeof(C), c->stream, BM_ARGS(NRV))
  // rows in blocks of at most 8 (one launch each)
  for (int rb = 0; rb < nr; rb += 8) {
    const int nrl = std::min(8, nr - rb);
    const bool lds = (size_t)d.n_b * (8 + BML_GROUPS(4) * 4) * sizeof(C) <= BM_LDS_MAX;
    if constexpr (sizeof(T) == 4) {
      if (lds) {
        if (nrl <= 4) BML(4, 4);
        else BML(8, 4);
      } else {
        if (nrl <= 4) BM(4, 4);
        else BM(8, 4);
      }
    } else {
      if (lds) {
        if (nrl <= 4) BML(4, 2);
        else BML(8, 2);
      } else {
        if (nrl <= 4) BM(4, 4);
        else BM(8, 2);
      }
    }
  }
#undef BML
#undef BM
#undef BM_ARGS
#undef BML_GROUPS
#undef BML_GRID
#undef BML_WGK
#undef BM_GRID
}

int run_build_M(lrigw_ctx *c, int iq, int slice, const void *H, const void *evec, void *M_out) {
  const Dims &d = c->d;
  int r0, nr, c0, nc;
  const int *kmap;
  if (slice == 0) {
    r0 = 0; nr = d.n_occ; c0 = d.n_occ; nc = d.n_unocc; kmap = c->d_kpq;
  } else if (slice == 1) {
    r0 = d.qp_lo; nr = d.n_qp; c0 = 0; nc = d.n_bands; kmap = c->d_kmq;
  } else {
    r0 = d.qp_lo; nr = d.n_qp; c0 = 0; nc = d.n_occ; kmap = c->d_kmq;
  }
  if (c->precision == LRIGW_FP64) launch_build<double>(c, iq, r0, nr, c0, nc, kmap, H, evec, M_out);
  else launch_build<float>(c, iq, r0, nr, c0, nc, kmap, H, evec, M_out);
  return lrigw_launch_check("build_M");
}

// ---------------------------------------------------------------- q = 0 preparation
// Dominant eigenpair of a Hermitian positive definite matrix by power
// iteration (one workgroup, x and V x in LDS).  Stops when
// ||V x - lambda x|| <= 1e-13 lambda; status[0] = iterations or -1.
__global__ __launch_bounds__(1024) void k_power_iter(const double2 *__restrict__ V, int n, int max_it, double2 *__restrict__ x_out,
                                                     double *__restrict__ lam_out, int *__restrict__ status) {
  extern __shared__ double2 sm[];
  double2 *x = sm;
  double2 *y = sm + n;
  __shared__ double red[32];
  __shared__ double bcast[4];
  __shared__ int istart;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) {
    double best = -1.0;
    int bi = 0;
    for (int i = 0; i < n; ++i)
      if (V[(long long)i * n + i].x > best) { best = V[(long long)i * n + i].x; bi = i; }
    istart = bi;
  }
  __syncthreads();
  // start from the column of the largest diagonal element
  for (int i = tid; i < n; i += blockDim.x) x[i] = V[(long long)i * n + istart];
  __syncthreads();
  auto block_sum = [&](double v) -> double {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
  };
  double nrm = 0.0;
  for (int i = tid; i < n; i += blockDim.x) nrm += x[i].x * x[i].x + x[i].y * x[i].y;
  nrm = sqrt(block_sum(nrm));
  for (int i = tid; i < n; i += blockDim.x) { x[i].x /= nrm; x[i].y /= nrm; }
  __syncthreads();
  int it = 0, done = 0;
  double lam = 0.0;
  for (it = 1; it <= max_it; ++it) {
    // y = V x, one wavefront per row
    for (int i = wv; i < n; i += nw) {
      double sr = 0.0, si = 0.0;
      const double2 *row = V + (long long)i * n;
      for (int j = lane; j < n; j += 64) {
        double2 v = row[j], xv = x[j];
        sr += v.x * xv.x - v.y * xv.y;
        si += v.x * xv.y + v.y * xv.x;
      }
      for (int o = 32; o > 0; o >>= 1) { sr += __shfl_xor(sr, o); si += __shfl_xor(si, o); }
      if (lane == 0) y[i] = mkc(sr, si);
    }
    __syncthreads();
    double l = 0.0;
    for (int i = tid; i < n; i += blockDim.x) l += x[i].x * y[i].x + x[i].y * y[i].y;  // Re x^H y
    lam = block_sum(l);
    double r2 = 0.0, y2 = 0.0;
    for (int i = tid; i < n; i += blockDim.x) {
      double dr = y[i].x - lam * x[i].x, di = y[i].y - lam * x[i].y;
      r2 += dr * dr + di * di;
      y2 += y[i].x * y[i].x + y[i].y * y[i].y;
    }
    r2 = block_sum(r2);
    y2 = block_sum(y2);
    double ny = sqrt(y2);
    for (int i = tid; i < n; i += blockDim.x) { x[i].x = y[i].x / ny; x[i].y = y[i].y / ny; }
    __syncthreads();
    if (sqrt(r2) <= 1e-13 * fabs(lam)) { done = 1; break; }
  }
  // final Rayleigh quotient with the normalised vector, and the phase convention
  for (int i = wv; i < n; i += nw) {
    double sr = 0.0, si = 0.0;
    const double2 *row = V + (long long)i * n;
    for (int j = lane; j < n; j += 64) {
      double2 v = row[j], xv = x[j];
      sr += v.x * xv.x - v.y * xv.y;
      si += v.x * xv.y + v.y * xv.x;
    }
    for (int o = 32; o > 0; o >>= 1) { sr += __shfl_xor(sr, o); si += __shfl_xor(si, o); }
    if (lane == 0) y[i] = mkc(sr, si);
  }
  __syncthreads();
  double l = 0.0;
  for (int i = tid; i < n; i += blockDim.x) l += x[i].x * y[i].x + x[i].y * y[i].y;
  lam = block_sum(l);
  if (tid == 0) {
    double best = -1.0;
    int bi = 0;
    for (int i = 0; i < n; ++i) {
      double m = x[i].x * x[i].x + x[i].y * x[i].y;
      if (m > best) { best = m; bi = i; }
    }
    double a = sqrt(best);
    bcast[0] = x[bi].x / a;   // e^{i phi} of the largest component
    bcast[1] = x[bi].y / a;
  }
  __syncthreads();
  const double pr = bcast[0], pi = bcast[1];
  for (int i = tid; i < n; i += blockDim.x) {
    double2 v = x[i];
    x_out[i] = mkc(v.x * pr + v.y * pi, v.y * pr - v.x * pi);  // x * conj(phase)
  }
  if (tid == 0) {
    lam_out[0] = lam;
    status[0] = done ? it : -1;
  }
}

int run_gamma_prepare(lrigw_ctx *c, const void *Vcut0, const void *p, double omega_cell) {
  const Dims &d = c->d;
  const int n = d.n_aux;
  if ((size_t)2 * n * sizeof(double2) > 140 * 1024) return LRIGW_ERR_ARG;
  double *dlam = nullptr;
  LRIGW_HIP_TRY(hipFuncSetAttribute((const void *)k_power_iter, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(2 * n * sizeof(double2))));
  LRIGW_HIP_TRY(hipMalloc(&dlam, sizeof(double)));
  hipLaunchKernelGGL(k_power_iter, dim3(1), dim3(1024), 2 * n * sizeof(double2), c->stream, (const double2 *)Vcut0, n, 5000,
                     c->d_x1, dlam, c->d_info);
  int rc = lrigw_launch_check("power_iter");
  double lam = 0.0;
  int st = -1;
  if (rc == LRIGW_OK) {
    hipMemcpyAsync(&lam, dlam, sizeof(double), hipMemcpyDeviceToHost, c->stream);
    hipMemcpyAsync(&st, c->d_info, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = lrigw_hip_error(e, "power_iter sync", __FILE__, __LINE__);
  }
  (void)hipFree(dlam);
  if (rc < 0) return rc;
  if (st < 0 || !(lam > 0.0)) return LRIGW_ERR_NOCONV;
  c->v1 = lam;
  c->gamma_p = p;
  c->omega_cell = omega_cell;
  if (!c->d_bhat) LRIGW_HIP_TRY(hipMalloc(&c->d_bhat, (size_t)lrigw_K(c) * d.n_aux * lrigw_csize(c)));
  c->gamma_ready = true;
  return LRIGW_OK;
}

// B^[K] = B[K] + X1 (y_K / sqrt(v1) - X1^H B[K]),  y_K = sqrt(4 pi / Omega) p_K / D_K.
// One wavefront per K; the projection is accumulated in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_gamma_modify(const typename c2t<T>::type *__restrict__ B, const double2 *__restrict__ x1,
                                                      const double2 *__restrict__ p, const T *__restrict__ delta, long long K,
                                                      int n, double yscale, typename c2t<T>::type *__restrict__ Bh) {
  typedef typename c2t<T>::type C;
  const long long Kidx = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (Kidx >= K) return;
  const C *b = B + Kidx * n;
  double sr = 0.0, si = 0.0;
  for (int m = lane; m < n; m += 64) {
    double2 xv = x1[m];
    double2 bv = to_z(b[m]);
    sr += xv.x * bv.x + xv.y * bv.y;  // conj(x) b
    si += xv.x * bv.y - xv.y * bv.x;
  }
  for (int o = 32; o > 0; o >>= 1) { sr += __shfl_xor(sr, o); si += __shfl_xor(si, o); }
  const double dl = (double)delta[Kidx];
  const double2 pk = p[Kidx];
  const double cr = yscale * pk.x / dl - sr, ci = yscale * pk.y / dl - si;
  C *o = Bh + Kidx * n;
  for (int m = lane; m < n; m += 64) {
    double2 xv = x1[m];
    double2 bv = to_z(b[m]);
    o[m] = to_c<T>(mkc(bv.x + xv.x * cr - xv.y * ci, bv.y + xv.x * ci + xv.y * cr));
  }
}

// D[K] = e_a(k+q) - e_i(k), K = (k * n_occ + i) * n_unocc + a
template <typename T>
__global__ void k_delta(const double *__restrict__ eig, const int *__restrict__ kpq, int iq, int nk, int n_bands, int n_occ,
                        int n_unocc, T *__restrict__ delta) {
  long long K = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long tot = (long long)nk * n_occ * n_unocc;
  if (K >= tot) return;
  int a = (int)(K % n_unocc);
  int i = (int)((K / n_unocc) % n_occ);
  int k = (int)(K / ((long long)n_unocc * n_occ));
  int k2 = kpq[k * nk + iq];
  delta[K] = (T)(eig[(long long)k2 * n_bands + n_occ + a] - eig[(long long)k * n_bands + i]);
}

int launch_delta(lrigw_ctx *c, int iq, const double *eig) {
  const Dims &d = c->d;
  long long K = lrigw_K(c);
  dim3 grid((unsigned)((K + 255) / 256));
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_delta<double>, grid, dim3(256), 0, c->stream, eig, c->d_kpq, iq, d.n_k, d.n_bands, d.n_occ, d.n_unocc,
                       (double *)c->d_delta);
  else
    hipLaunchKernelGGL(k_delta<float>, grid, dim3(256), 0, c->stream, eig, c->d_kpq, iq, d.n_k, d.n_bands, d.n_occ, d.n_unocc,
                       (float *)c->d_delta);
  return lrigw_launch_check("delta");
}

int launch_gamma_modify(lrigw_ctx *c, const void *B) {
  const Dims &d = c->d;
  long long K = lrigw_K(c);
  double ys = sqrt(4.0 * M_PI / c->omega_cell) / sqrt(c->v1);
  dim3 grid((unsigned)((K + 3) / 4));
  if (c->precision == LRIGW_FP64)
    hipLaunchKernelGGL(k_gamma_modify<double>, grid, dim3(256), 0, c->stream, (const double2 *)B, c->d_x1,
                       (const double2 *)c->gamma_p, (const double *)c->d_delta, K, d.n_aux, ys, (double2 *)c->d_bhat);
  else
    hipLaunchKernelGGL(k_gamma_modify<float>, grid, dim3(256), 0, c->stream, (const float2 *)B, c->d_x1,
                       (const double2 *)c->gamma_p, (const float *)c->d_delta, K, d.n_aux, ys, (float2 *)c->d_bhat);
  return lrigw_launch_check("gamma_modify");
}
