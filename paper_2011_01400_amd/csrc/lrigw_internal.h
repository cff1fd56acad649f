// Internal declarations of the lrigw HIP library (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/lrigw.h"

// ---------------------------------------------------------------- complex helpers
template <typename T> struct c2t;
template <> struct c2t<double> { typedef double2 type; };
template <> struct c2t<float> { typedef float2 type; };

__host__ __device__ inline double2 mkc(double r, double i) { double2 z; z.x = r; z.y = i; return z; }
__host__ __device__ inline float2 mkcf(float r, float i) { float2 z; z.x = r; z.y = i; return z; }
template <typename C> __host__ __device__ inline C cmul(C a, C b) { C z; z.x = a.x * b.x - a.y * b.y; z.y = a.x * b.y + a.y * b.x; return z; }
template <typename C> __host__ __device__ inline C cconj(C a) { a.y = -a.y; return a; }
template <typename C> __host__ __device__ inline C cadd(C a, C b) { a.x += b.x; a.y += b.y; return a; }
// p[i] if ok, else z: the load always happens (from index 0 when !ok, which
// must be valid), so a run of these issues all its loads before any wait; a
// branch around each load would serialise them
template <typename V> __device__ inline V ld_or(const V *__restrict__ p, long long i, bool ok, V z) {
  const V v = p[ok ? i : 0];
  return ok ? v : z;
}
// a * conj(b)
template <typename C> __host__ __device__ inline C cmulc(C a, C b) { C z; z.x = a.x * b.x + a.y * b.y; z.y = a.y * b.x - a.x * b.y; return z; }
// conj(a) * b
template <typename C> __host__ __device__ inline C ccmul(C a, C b) { C z; z.x = a.x * b.x + a.y * b.y; z.y = a.x * b.y - a.y * b.x; return z; }

template <typename T> __device__ inline typename c2t<T>::type to_c(double2 z);
template <> __device__ inline double2 to_c<double>(double2 z) { return z; }
template <> __device__ inline float2 to_c<float>(double2 z) { return mkcf((float)z.x, (float)z.y); }
__device__ inline double2 to_z(double2 z) { return z; }
__device__ inline double2 to_z(float2 z) { return mkc(z.x, z.y); }

// ---------------------------------------------------------------- error plumbing
#define LRIGW_HIP_TRY(expr)                                   \
  do {                                                        \
    hipError_t e__ = (expr);                                  \
    if (e__ != hipSuccess) return lrigw_hip_error(e__, #expr, __FILE__, __LINE__); \
  } while (0)
#define LRIGW_TRY(expr)                \
  do {                                 \
    int r__ = (expr);                  \
    if (r__ < 0) return r__;           \
  } while (0)

int lrigw_hip_error(hipError_t e, const char *what, const char *file, int line);
int zero_fill(hipStream_t s, void *p, size_t bytes);
int lrigw_launch_check(const char *what);

// ---------------------------------------------------------------- context
struct Dims {
  int n_atoms = 0, n_k = 0, nk[3] = {1, 1, 1};
  int n_b = 0, n_aux = 0, n_bands = 0, n_occ = 0, n_unocc = 0;
  int n_freq = 0, qp_lo = 0, n_qp = 0, nb_max = 0;
  double x0 = 0.5, mu = 0.0;
};

struct StageTimer {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  double ms = 0.0;
  long long launches = 0;
};

struct lrigw_ctx {
  Dims d;
  int precision = LRIGW_FP64;
  int device = 0;                // HIP device current at lrigw_create
  hipStream_t stream = nullptr;
  std::vector<int> basis_off, aux_off;
  std::vector<int> h_kpq, h_kmq;

  // device tables
  int *d_aux_atom = nullptr;     // [N_aux] atom of each auxiliary function
  int *d_basis_off = nullptr;    // [n_atoms+1]
  int *d_aux_off = nullptr;      // [n_atoms+1]
  int *d_kpq = nullptr, *d_kmq = nullptr;
  double *d_omega = nullptr, *d_weight = nullptr;
  int *d_wall = nullptr;         // [N_w] 0, 1, ..., N_w - 1 (every frequency selected)
  std::vector<double> h_omega, h_weight;
  // per-plane tables of the response kernels, [2 N_w]: the imaginary planes,
  // then the real-axis planes.  om2 is the signed square (+w^2 on the
  // imaginary axis, -w^2 on the real axis, so the weight 2D/(D^2 + om2) is
  // the one of either axis); wsc the FP16 split's power-of-two weight scale.
  double *d_om2 = nullptr;
  float *d_wsc = nullptr;
  std::vector<double> h_om2;
  std::vector<float> h_wsc;
  double gap_min = 0.0;          // smallest transition energy of the checked eigenvalues
  double gap_max = 0.0;          // largest transition energy of the checked eigenvalues
  // real-axis grid w_r = r h, r < n_real (0: none); its buffers
  int n_real = 0;
  // broadened real grid (real_eta > 0): W^c at w_r + i eta for every w_r, the
  // response from two weight planes per node (tables of 2 n_real planes: node
  // r's Re part at 2r, Im part at 2r+1)
  double real_eta = 0.0;
  double *d_bom2 = nullptr;      // [2 n_real] eta^2 - w_r^2
  double2 *d_bcpl = nullptr;     // [2 n_real] (2 w_r eta, part)
  float *d_bwsc = nullptr;       // [2 n_real] FP16 weight scales
  std::vector<float> h_bwsc;
  double bwsc_gap = -1.0, bwsc_gmax = -1.0;   // transition window the scales were made for
  double real_h = 0.0, real_wsc_gap = -1.0;
  void *d_chir = nullptr, *d_wr = nullptr;   // [n_real][N][N] response / W^c (compute type)
  void *d_chir2 = nullptr, *d_wr2 = nullptr; // second pair (the pass screens q while building q+1)
  double *d_Xr = nullptr;        // [n_real][N_k*n_qp*n_bands] pair weights on the real grid
  double *d_cdE = nullptr;       // [3][N_k][n_qp] evaluation energies of the linearised QP
  double *d_cdS = nullptr;       // [3][N_k][n_qp] Sigma^c at those energies
  int *d_cdbad = nullptr;        // count of (e, k, n) whose residues passed the grid's top

  // per-q workspaces
  void *d_delta = nullptr;       // [K] transition energies of one q (T)
  void *d_part = nullptr;        // chi0 split-K partials
  size_t part_bytes = 0;
  int chi_splits = 1;
  int chi_nw = 4;                // frequencies per chi0 workgroup
  int chi_pad = 8;               // split-BF16 chi0: LDS row padding (BF16 elements)
  int sig_var = 0;               // split-BF16 Sigma^c kernel variant
  void *d_X = nullptr;           // [N_w][N_k*n_qp*n_bands] pair weights (T)
  double2 *d_LV = nullptr;       // [N][N]
  double2 *d_cut = nullptr;      // truncated-Coulomb screening: L^{-1} V^{1/2} V^cut^{1/2} and workspace (13 N^2)
  // Coulomb factors of a whole pass (CoulombScope): L(q) with V(q) = L L^H and,
  // with V^cut, T^H(q) = L^{-1} V^{1/2} V^cut^{1/2}, for q in [cf_q0, cf_q1)
  double2 *d_cf = nullptr;       // [L(q) ...][T^H(q) ...][diagonal-block inverses][root workspace]
  // grouped screening (run_pass without graph capture): the responses and
  // W^c of up to grp_cap q, FP64 workspaces and diagonal-block inverses
  void *d_grp = nullptr;
  size_t grp_bytes = 0;
  int grp_cap = 0;
  size_t cf_bytes = 0;
  const void *cf_V = nullptr, *cf_Vcut = nullptr;
  int cf_q0 = 0, cf_q1 = 0;
  bool cf_on = false, cf_cut = false;
  double2 *d_s0 = nullptr, *d_s1 = nullptr, *d_s2 = nullptr, *d_s3 = nullptr;  // [N_w][N][N]
  double2 *d_dinv = nullptr;     // inverses of 64x64 diagonal Cholesky blocks, [N_w][zdinv_stride(N)]
  int *d_info = nullptr;         // device status words
  void *d_bhat = nullptr;        // q = 0 modified B (T)
  void *d_ap = nullptr;          // split-BF16 forms: BF16 parts of B, [NS][2][Npad][Kp] (k contiguous)
  void *d_bt = nullptr;          // split forms: B transposed (FP16 split: row-scaled), FP32 [Npad][Kp]
  void *d_xs = nullptr;          // split forms: 16-bit parts of conj(x), [NS][2][Cpad][Npad]
  void *d_ws = nullptr;          // split forms: 16-bit parts of lower W^c, [N_w][NS][2][Rpad][Npad]
  float *d_sx = nullptr;         // FP16 split: power-of-two scale of each x column [Cpad]
  unsigned *d_wmax = nullptr;    // FP16 split: largest |W^c(w)| as float bits [N_w]
  unsigned *d_amax = nullptr;    // FP16 split: largest |B| of each auxiliary row as float bits [Rpad]
  int *d_sitems = nullptr;       // resident-tile Sigma^c form: per-wave item lists
  double *d_wd = nullptr;        // resident-tile Sigma^c form: Re W^c_mumu(w), [N_aux][32]
  void *d_xo = nullptr;          // exchange pairs of one q (build_M slice 2), compute type
  void *d_sxa = nullptr;         // the same pairs in FP64 (reduced-precision forms)
  void *d_sxz = nullptr;         // V x of those pairs, FP64
  int sig_res_F = 0;             // resident-tile Sigma^c form: frequencies per workgroup
  int sig_res_F4 = 0;            // the same with four frequency sets (eight waves; 0: no plan)
  bool sig_res_ok = false;       // resident-tile Sigma^c form applies to this cell
  int *d_sitems_r = nullptr;     // resident-tile form: item lists for the real-axis planes (contour deformation)
  int sig_res_Fr = 0, sig_res_nr = 0;   // their frequencies per workgroup and plane count (0: no plan)
  int sig_res_Fr4 = 0;           // the same with four frequency sets

  // q = 0 data
  double2 *d_x1 = nullptr;       // [N_aux]
  double v1 = 0.0;
  const void *gamma_p = nullptr;
  double omega_cell = 0.0;
  bool gamma_ready = false;
  // q -> 0 averaged over directions (n_gdir = 0: the single direction gamma_p)
  int n_gdir = 0;
  const void *gdir_p = nullptr;  // caller's complex128 [n_gdir][N_k][n_occ][n_unocc], p . q_hat_d
  std::vector<double> gdir_w;

  // driver-owned buffers (chi and W^c double buffered: the screening of q runs
  // on stream2 while the response of q+1 is built on stream)
  void *d_M = nullptr, *d_x = nullptr, *d_chi = nullptr, *d_wc = nullptr;
  void *d_chi2 = nullptr, *d_wc2 = nullptr;
  hipStream_t stream2 = nullptr;
  hipEvent_t ev_chi[2] = {nullptr, nullptr}, ev_wc[2] = {nullptr, nullptr};

  // > 0 while a whole pass (or a captured graph) runs whose eigenvalues were
  // checked for a gap at its start: the per-q response calls skip the check
  int gap_trusted = 0;

  // graph capture: no host round trips; screening status folded into d_info[16]
  bool capturing = false;
  double *d_epsqp = nullptr;     // [N_k][n_qp] band energies of the QP bands (driver)

  // learned frequency surrogate used by the driver (not owned)
  lrigw_surrogate *sur = nullptr;
  double sur_threshold = 0.0;

  // timing
  int timing = 0;   // 0 off, 1 every stage, 2 the two MFMA kernel stages only
  std::map<std::string, StageTimer> stages;
};

size_t lrigw_csize(const lrigw_ctx *c);   // bytes of one complex T
// marks the eigenvalues as checked for the lifetime of the scope
struct GapScope {
  lrigw_ctx *c;
  explicit GapScope(lrigw_ctx *ctx) : c(ctx) { ++c->gap_trusted; }
  ~GapScope() { --c->gap_trusted; }
  GapScope(const GapScope &) = delete;
  GapScope &operator=(const GapScope &) = delete;
};
// Factors V(q) = L L^H (and the V^cut factors) of q in [q0, q1) for a whole
// pass at once, batched over q, on the context stream; while the scope lives
// the screening takes them when called with V + q N^2 (and V^cut + q N^2 for
// q > 0).  A V(q) that is not positive definite marks d_info[16] with its q.
// Not used during graph capture (no allocation there): then each screening
// factors its own V(q).
int coulomb_factors(lrigw_ctx *c, const void *V, const void *Vcut, int q0, int q1);
// Screening of the nq consecutive q from q0 at once (batch nq N_w), with the
// factors of the live CoulombScope (which must cover them): chi and Wc_out
// hold nq blocks of N_w planes; ws: FP64 workspace of group_ws_elems(c, nq)
// complex elements.  Status as in a pass (d_info[16] = first failing q).
int run_screen_group(lrigw_ctx *c, int q0, int nq, const void *chi, const void *V, const void *Vcut, void *Wc_out,
                     double2 *ws);
long long group_ws_elems(const lrigw_ctx *c, int nq);
struct CoulombScope {
  lrigw_ctx *c;
  explicit CoulombScope(lrigw_ctx *ctx) : c(ctx) {}
  ~CoulombScope() { c->cf_on = false; }
  CoulombScope(const CoulombScope &) = delete;
  CoulombScope &operator=(const CoulombScope &) = delete;
};
// BF16 parts of the response / self-energy operands (0: not a split form)
inline int ns_chi(int precision) {
  return (precision == LRIGW_SPLIT_BF16 || precision == LRIGW_SPLIT_MIXED || precision == LRIGW_SPLIT_F16) ? 2
         : precision == LRIGW_SPLIT3_BF16                                                                 ? 3
                                                                                                          : 0;
}
inline int ns_sig(int precision) {
  return (precision == LRIGW_SPLIT_BF16 || precision == LRIGW_SPLIT_F16)        ? 2
         : (precision == LRIGW_SPLIT3_BF16 || precision == LRIGW_SPLIT_MIXED) ? 3
                                                                             : 0;
}
// split parts are FP16 (scaled) rather than BF16
inline bool split_h(int precision) { return precision == LRIGW_SPLIT_F16; }
long long lrigw_K(const lrigw_ctx *c);    // N_k * n_occ * n_unocc

// stage timing helpers (no-ops unless timing is on)
void stage_begin(lrigw_ctx *c, const char *name, hipEvent_t *ev);
void stage_end(lrigw_ctx *c, const char *name, hipEvent_t ev);

// ---------------------------------------------------------------- kernel entry points (host side)
int run_grids(lrigw_ctx *c);
int chi0_default_nw(int precision);
int chi0_alt_nw(int precision);
int chi0_plan_splits(const lrigw_ctx *c, int *splits);
size_t chi0_part_bytes(const lrigw_ctx *c, int splits);
// split forms: the longest K chunk one workgroup may sum in FP32 (the tuner
// and lrigw_set_tiles keep splits >= ceil(K / CHI0_SPLIT_MAX_ROWS))
#define CHI0_SPLIT_MAX_ROWS 4096
inline long long chi0_min_splits(const lrigw_ctx *c, long long K) {
  return ns_chi(c->precision) > 0 ? (K + CHI0_SPLIT_MAX_ROWS - 1) / CHI0_SPLIT_MAX_ROWS : 1;
}
int chi0_check_gap(lrigw_ctx *c, const double *eig);
int sigma_variant_snw(int var);
int sigma_variants();
bool sigma_variant_ok(const lrigw_ctx *c, int var);
int sigma_res_prepare(lrigw_ctx *c);
int sigma_default_variant(int precision);
int run_lri_ft(lrigw_ctx *c, const double *lri_R, const int *R_list, int nR, const void *evec, void *H_out);
int run_build_M(lrigw_ctx *c, int iq, int slice, const void *H, const void *evec, void *M_out);
int run_chi0(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out);
int run_chi0_sel(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out, const int *wsel,
                 int n_sel, const int *run, bool real_axis = false);
// per-plane tables of the response kernels (device): signed w^2 (weight
// 2D/(D^2 + om2)), the FP16 split's weight scale, and for complex-frequency
// planes (cpl != nullptr) (s, part): the Re (part 0) or Im part of
// 2D/(D^2 - z^2) with z^2 = -om2 + i s
struct PlaneTab {
  const double *om2;
  const float *wsc;
  const double2 *cpl;
};
int run_chi0_tab(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out, const int *wsel,
                 int n_sel, const int *run, const PlaneTab &tab);
int surrogate_prepare(lrigw_surrogate *sg);
int run_chi0_surrogate(lrigw_ctx *c, lrigw_surrogate *sg, int iq, const void *M, const double *eig, int apply_gamma,
                       double threshold, void *chi_out);
int run_gamma_prepare(lrigw_ctx *c, const void *Vcut0, const void *p, double omega_cell);
// Vcut: the truncated Coulomb matrix of the numerator (nullptr or V: V itself)
int run_screen(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info);
int run_screen_n(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wc_out, int *info, int nw);
int run_screen_cplx(lrigw_ctx *c, int iq, const void *chi, const void *V, const void *Vcut, void *Wh_out, int *info,
                    int np);
int run_sigma_c(lrigw_ctx *c, int iq, const void *x, const void *Wc, const double *eig, void *sigma_acc);
int run_pair_weights(lrigw_ctx *c, const void *x, const void *Wc, int nw, double *X);
int sigma_res_prepare_real(lrigw_ctx *c, int n_r);
int run_set_real_grid(lrigw_ctx *c, int n_r, double omega_max, double eta);
int run_cd_pass_broadened(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V,
                          const void *Vcut, const void *p, double omega_cell, int n_e, const double *E, double *sigma_e,
                          int *n_bad);
int cd_newton(lrigw_ctx *c, const double *eig, const double *S, const double *e_static, double delta, double *e_cur,
              double *z, int first);
int run_chi0_real(lrigw_ctx *c, int iq, const void *M, const double *eig, int apply_gamma, void *chi_out);
int run_sigma_cd(lrigw_ctx *c, int iq, const void *x, const void *Wc, const void *Wr, const double *eig, int n_e,
                 const double *E, double *sigma_e);
int cd_energies(lrigw_ctx *c, const double *eig, double delta);
int cd_qp_linear(lrigw_ctx *c, const double *S, const double *e_static, double delta, double *e_qp, double *z);
int cd_count_nan(lrigw_ctx *c, const double *v, int n, int *out);
int run_pade_eval(lrigw_ctx *c, const void *sigma, int n_par, int n_e, const double *E, void *out);
int run_gamma_average(lrigw_ctx *c, const double *eig, const void *V0, bool real_axis, void *chi, void *tmp, void *out);
int run_cd_pass(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
                const void *p, double omega_cell, int n_e, const double *E, double *sigma_e, int *n_bad);
int run_sigma_x(lrigw_ctx *c, int iq, const void *xo, const void *V, double *sigma_x);
int run_lri_fit(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T, double scale,
                double *C, int *info);
// allocation-free fit: workspace in a fixed per-device array of LRIGW_FIT_SCRATCH_BYTES
#define LRIGW_MAX_DEVICES 64
int fit_scratch_prepare(int dev);
size_t fit_scratch_bytes(int batch, int n, int nrhs);
int run_lri_fit_noalloc(lrigw_ctx *c, int batch, int n, int n_keep, int nrhs, const double *V, const double *T,
                        double scale, double *C, int *info);
int run_pass(lrigw_ctx *c, const void *H, const void *evec, const double *eig, const void *V, const void *Vcut,
             const void *p, double omega_cell, const double *e_static, int n_par, int q_first, int q_last, void *sigma,
             double *e_qp, double *z, int *info);
int driver_buffers(lrigw_ctx *c);
int run_qp(lrigw_ctx *c, const void *sigma, const double *eps_qp, const double *e_static, int n_par, double *e_qp,
           double *z, int *info);

// dense FP64 complex helpers (k_dense.hip)
enum { OP_N = 0, OP_T = 1, OP_C = 2 };
struct ZGemm {
  int m, n, k;
  int opa, opb;
  const double2 *A; long long lda, sa;    // sa: batch stride (elements)
  const double2 *B; long long ldb, sb;
  double2 *C; long long ldc, sc;
  double2 alpha, beta;
  int batch;
  int lower_only;                          // skip tiles strictly above the diagonal
  // op(A) / op(B) triangular with zeros stored in the other triangle (TRI_LOWER,
  // TRI_UPPER): each tile then runs only the K range its rows / columns need
  int tri_a = 0, tri_b = 0;
  // batch element b reads A at (b % bdiv) sa + (b / bdiv) sa2 (and B alike):
  // one operand per group of bdiv elements (a factor per q for its frequencies)
  int bdiv = 1 << 30;
  long long sa2 = 0, sb2 = 0;
};
enum { TRI_NONE = 0, TRI_LOWER = 1, TRI_UPPER = 2 };
int zgemm(hipStream_t s, const ZGemm &g);
long long zdinv_stride(int n);
int zpotrf_batched(hipStream_t s, double2 *A, int n, long long lda, long long stride, int batch, double2 *Dinv, int *d_info);
int ztrsm_left_lower(hipStream_t s, const double2 *L, long long ldl, long long sl, const double2 *Dinv, double2 *Y,
                     long long ldy, long long sy, int n, int ncols, int batch);
int ztrsm_left_upper_conj(hipStream_t s, const double2 *L, long long ldl, long long sl, const double2 *Dinv, double2 *Y,
                          long long ldy, long long sy, int n, int ncols, int batch);
