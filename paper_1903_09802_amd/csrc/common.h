// Internal declarations shared by the HIP sources of the DDA library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <string>
#include <vector>

#include "../../include/dda.h"

// ----------------------------------------------------------------------------- complex helpers

template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };
template <typename T> using cplx = typename C2<T>::type;

template <typename T> __host__ __device__ __forceinline__ cplx<T> mk(T re, T im) {
  cplx<T> r; r.x = re; r.y = im; return r;
}
template <typename V> __host__ __device__ __forceinline__ V cadd(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __host__ __device__ __forceinline__ V csub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V> __host__ __device__ __forceinline__ V cmul(V a, V b) {
  V r; r.x = a.x * b.x - a.y * b.y; r.y = a.x * b.y + a.y * b.x; return r;
}
// conj(a) * b
template <typename V> __host__ __device__ __forceinline__ V cmulcj(V a, V b) {
  V r; r.x = a.x * b.x + a.y * b.y; r.y = a.x * b.y - a.y * b.x; return r;
}
template <typename V, typename S> __host__ __device__ __forceinline__ V cscale(V a, S s) { V r; r.x = a.x * s; r.y = a.y * s; return r; }
template <typename V> __host__ __device__ __forceinline__ V cconj(V a) { V r; r.x = a.x; r.y = -a.y; return r; }
// acc + a b as four fused multiply-adds
template <typename V> __host__ __device__ __forceinline__ V cmac(V acc, V a, V b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
// multiply by -i (sign = -1) or +i (sign = +1)
template <typename V> __host__ __device__ __forceinline__ V cmuli(V a, int sign) {
  V r; if (sign > 0) { r.x = -a.y; r.y = a.x; } else { r.x = a.y; r.y = -a.x; } return r;
}
__host__ __device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  double den = b.x * b.x + b.y * b.y;
  return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}
template <typename V> __device__ __forceinline__ V ldc(const V *p) { return *p; }

// Workgroups are dealt to the 8 XCDs (each with its own L2) round robin.  A kernel that
// launches xcd_grid(G) blocks and maps blockIdx through xcd_remap gets logically adjacent
// work items (which share cache lines) on the same XCD; indices >= G exit at once.
constexpr int kXcds = 8;
// Largest Krylov basis (restart + 1 vectors); per-RHS arrays of small vectors use this stride.
// 1024 lets GMRES keep the whole Krylov space for the few hundred iterations the paper's
// hardest converging cases need (Sec. 4); the basis and the Gram matrix are sized by the
// actual restart.
constexpr int kMaxM = 1024;
__host__ __device__ __forceinline__ long long xcd_grid(long long G) {
  return ((G + kXcds - 1) / kXcds) * kXcds;
}
__device__ __forceinline__ long long xcd_remap(long long b, long long G) {
  const long long per = (G + kXcds - 1) / kXcds;
  return (b % kXcds) * per + b / kXcds;
}

__device__ __forceinline__ float2 to_c(double2 a, float2) { return make_float2((float)a.x, (float)a.y); }
__device__ __forceinline__ double2 to_c(double2 a, double2) { return a; }
__device__ __forceinline__ double2 to_d(float2 a) { return make_double2((double)a.x, (double)a.y); }
__device__ __forceinline__ double2 to_d(double2 a) { return a; }

// LDR polarisability coefficients (Sec. 2.1) and its inverse with the voxel volume omitted:
// 1/alpha = (4 pi / 3)(eps + 2)/(eps - 1) + (b1 + eps b2 + eps b3 S)(k d)^2 - (2i/3)(k d)^3.
#define DDA_B1 (-1.891531)
#define DDA_B2 (0.1648469)
#define DDA_B3 (-1.7700004)
#define DDA_PI 3.14159265358979323846

__host__ __device__ __forceinline__ double2 ldr_alpha_inv(double2 eps, double kd, double S) {
  double2 num = make_double2(eps.x + 2.0, eps.y);
  double2 den = make_double2(eps.x - 1.0, eps.y);
  double2 q = cdiv(num, den);
  double f = 4.0 * DDA_PI / 3.0;
  double kd2 = kd * kd;
  double2 r;
  r.x = f * q.x + (DDA_B1 + eps.x * (DDA_B2 + DDA_B3 * S)) * kd2;
  r.y = f * q.y + eps.y * (DDA_B2 + DDA_B3 * S) * kd2 - (2.0 / 3.0) * kd2 * kd;
  return r;
}
// The same with the Clausius-Mossotti ratio q = (eps + 2)/(eps - 1) given: 1/alpha is linear in
// eps apart from q, so the mean of 1/alpha over voxels is this at the means of q and eps.
__host__ __device__ __forceinline__ double2 ldr_alpha_inv_q(double2 q, double2 eps, double kd, double S) {
  const double f = 4.0 * DDA_PI / 3.0;
  const double kd2 = kd * kd;
  double2 r;
  r.x = f * q.x + (DDA_B1 + eps.x * (DDA_B2 + DDA_B3 * S)) * kd2;
  r.y = f * q.y + eps.y * (DDA_B2 + DDA_B3 * S) * kd2 - (2.0 / 3.0) * kd2 * kd;
  return r;
}
// d(1/alpha)/d eps = -4 pi / (eps - 1)^2 + (b2 + b3 S)(k d)^2
__host__ __device__ __forceinline__ double2 ldr_dalpha_inv(double2 eps, double kd, double S) {
  double2 em1 = make_double2(eps.x - 1.0, eps.y);
  double2 sq = cmul(em1, em1);
  double2 t = cdiv(make_double2(-4.0 * DDA_PI, 0.0), sq);
  t.x += (DDA_B2 + DDA_B3 * S) * kd * kd;
  return t;
}

// Six unique tensor components, order xx, xy, xz, yy, yz, zz (Algorithm 1).
// Parity bit mask per component: bit a set when the component is odd under
// reflection of axis a (odd iff exactly one of its two indices is that axis).
__host__ __device__ __forceinline__ int comp_odd_mask(int c) {
  // xx:0, xy: x|y, xz: x|z, yy:0, yz: y|z, zz:0 (4 bits per component, no memory table)
  return (0x60530 >> (4 * c)) & 15;
}
__host__ __device__ __forceinline__ int comp_index(int a, int b) {
  // (a, b) -> xx 0, xy 1, xz 2, yy 3, yz 4, zz 5
  const int i = a < b ? a : b, j = a < b ? b : a;
  return 3 * i - (i * (i - 1)) / 2 + (j - i);
}

// ----------------------------------------------------------------------------- error handling

namespace dda {

void set_error(const char *fmt, ...);
const char *get_error();

struct Fail {
  dda_status st;
};

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      ::dda::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                        \
      throw ::dda::Fail{DDA_EDEVICE};                                                    \
    }                                                                                    \
  } while (0)

#define REQUIRE(cond, status, ...)        \
  do {                                    \
    if (!(cond)) {                        \
      ::dda::set_error(__VA_ARGS__);      \
      throw ::dda::Fail{status};          \
    }                                     \
  } while (0)

// ----------------------------------------------------------------------------- FFT plans

constexpr int kMaxRadices = 16;
constexpr int kMaxFft = 1024;

struct FftPlan {
  int n = 0;
  int nrad = 0;
  int rad[kMaxRadices] = {0};
  double2 *tw64 = nullptr;  // exp(-2 pi i t / n), t in [0, n)
  float2 *tw32 = nullptr;
};

// Device-side copy of a plan, passed by value to kernels.
struct FftDesc {
  int n;
  int nrad;
  int rad[kMaxRadices];
};

bool factor_7smooth(int n, FftPlan &plan);
void plan_create(FftPlan &plan, int n);
void plan_destroy(FftPlan &plan);
inline FftDesc desc(const FftPlan &p) {
  FftDesc d;
  d.n = p.n;
  d.nrad = p.nrad;
  for (int i = 0; i < kMaxRadices; ++i) d.rad[i] = p.rad[i];
  return d;
}

// ----------------------------------------------------------------------------- profiling

struct Profiler {
  bool on = false;
  std::string only;  // when not empty, only launches of this kind are timed
  struct Kind {
    std::string name;
    std::vector<float> ms;      // duration of every timed launch
    std::vector<double> bytes;  // its algorithmic bytes
    // launches that did work (a launch inside a finished solver cycle returns at once: under
    // 2 % of the kind's longest), their summed duration and algorithmic bytes
    void working(long long &n, double &total_ms, double &total_bytes) const;
  };
  std::vector<Kind> kinds;
  struct Pending {
    int kind;
    double bytes;
    hipEvent_t a, b;
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  int kind_id(const char *name);
  void begin(hipStream_t s, int kind, hipEvent_t *a, hipEvent_t *b);
  void collect();  // after a stream sync
  void reset();
  void destroy();
  hipEvent_t get_event();
};

// RAII timer around one launch; no-op when profiling is off.
// FFT passes whose tile shapes the autotuner picks (x rows and y columns of the operator and
// of the preconditioner), and a shape: columns per tile and, along a strided axis, tiles per
// workgroup (0: the launch rule).
enum FftPass {
  FP_OP_X_FWD, FP_OP_Y_FWD, FP_OP_Y_INV, FP_OP_X_INV,
  FP_PC_X_FWD, FP_PC_Y_FWD, FP_PC_Y_INV, FP_PC_X_INV, FP_COUNT
};
struct TileShape {
  int tw = 0, tpw = 0;
};

struct KTimer {
  Profiler *prof;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  KTimer(Profiler *p, hipStream_t s, const char *name, double bytes);
  ~KTimer();
};

}  // namespace dda

// ----------------------------------------------------------------------------- problem handle

// The library's frame: internal axis k (0 x', 1 y', 2 z') is the caller's axis ax[k], a
// cyclic rotation that puts the preconditioner's dense axis last; vector components rotate
// with the axes (internal component a is the caller's component ax[a]).  e* are the caller's
// dimensions, n* the internal ones (n_k = e_{ax[k]}).
struct Frame {
  int nx, ny, nz;
  int ex, ey;
  int ax0, ax1, ax2;
  // caller's voxel index of internal voxel v
  __host__ __device__ __forceinline__ long long to_ext(long long v) const {
    const long long i0 = v % nx, i1 = (v / nx) % ny, i2 = v / ((long long)nx * ny);
    const long long e0 = ax0 == 0 ? i0 : ax1 == 0 ? i1 : i2;
    const long long e1 = ax0 == 1 ? i0 : ax1 == 1 ? i1 : i2;
    const long long e2 = ax0 == 2 ? i0 : ax1 == 2 ? i1 : i2;
    return e0 + ex * (e1 + (long long)ey * e2);
  }
  // internal voxel index of the caller's voxel e
  __host__ __device__ __forceinline__ long long to_int(long long e) const {
    const long long e0 = e % ex, e1 = (e / ex) % ey, e2 = e / ((long long)ex * ey);
    const long long i0 = ax0 == 0 ? e0 : ax0 == 1 ? e1 : e2;
    const long long i1 = ax1 == 0 ? e0 : ax1 == 1 ? e1 : e2;
    const long long i2 = ax2 == 0 ? e0 : ax2 == 1 ? e1 : e2;
    return i0 + nx * (i1 + (long long)ny * i2);
  }
  // caller's component of internal component a, and the inverse
  __host__ __device__ __forceinline__ int comp_ext(int a) const { return a == 0 ? ax0 : a == 1 ? ax1 : ax2; }
  __host__ __device__ __forceinline__ int comp_int(int e) const { return ax0 == e ? 0 : ax1 == e ? 1 : 2; }
};

struct dda_problem {
  int nx = 0, ny = 0, nz = 0;
  Frame fr{};            // internal <-> caller's frame (identity for dense_axis 2)
  long long N = 0;       // voxels in the box
  long long n_occ = 0;   // occupied voxels
  double k = 0.0, d = 0.0;
  hipStream_t st = nullptr;
  dda_options opt{};
  int R = 1;             // max right-hand sides
  int dev = 0;           // the HIP device the handle lives on
  size_t lds_max = 65536;      // device LDS per workgroup
  size_t lds_zpass = 98304;    // LDS budget of the fused z pass
  int ztw[2] = {0, 0};         // z-pass columns per tile (FP64, FP32), chosen by autotune
  dda::TileShape tile[dda::FP_COUNT][2];  // x / y pass shapes per pass (FP64, FP32), chosen by autotune
  int zipw[2] = {0, 0};        // register z pass: forced items per workgroup (0: by the rule)
  int zreg = 0;                // 1: register z pass (2 nz = G P in its list of lengths); the
                               // kernel spectra are then stored z-major, [oy][ox][oz][6]

  uint8_t *mask = nullptr;      // [N]
  double2 *eps = nullptr;       // [N]
  // Field vectors inside the solver are compact, [R][3][nocc]: one entry per occupied voxel,
  // in voxel order.  cidx[v] is voxel v's entry (-1 in air), vox[c] the voxel of entry c.
  long long nocc = 0;
  int *cidx = nullptr;          // [N]
  int *vox = nullptr;           // [nocc]
  double2 eps_mean{0.0, 0.0};   // mean permittivity over occupied voxels
  double2 cm_mean{};            // mean over occupied voxels of (eps + 2) / (eps - 1)

  dda::FftPlan px, py, pz;   // padded lengths 2nx, 2ny, 2nz
  dda::FftPlan ux, uy;       // unpadded nx, ny (preconditioner)

  // operator kernel: FFT of the circulant embedding, octant [6][nz+1][ny+1][nx+1]
  double2 *khat64 = nullptr;
  float2 *khat32 = nullptr;
  double2 *khatI64 = nullptr;   // same for d^3 Im G (scattering sum)

  // FFT workspaces (sized for R right-hand sides, FP64 elements)
  void *w0 = nullptr;  // [R][3][nz][ny][2nx]
  void *w1 = nullptr;  // [R][3][nz][2ny][2nx]
  size_t w0_elems = 0, w1_elems = 0;
  long long zplane = 0;  // z-row stride of the z-pass work array w1 (4 nx ny plus padding)

  double2 *ainv = nullptr;   // [R][N] per-RHS 1/alpha
  double *Sdev = nullptr;    // [R] lattice factor per RHS

  // preconditioner
  int prec_built = 0;
  int prec_sweep = 0;          // 1: the last 2-level build inverted by the symmetric sweep
  int tune_xy = 0;             // 1 while the x / y tile tuner times its passes: the z pass and
                               // the block product, whose times do not enter, are not launched
  int prec_fp32 = 0;
  double2 ati{0.0, 0.0};     // alpha~^{-1}
  int pz0 = 0, pbz = 0;      // occupied z layers [pz0, pz0 + pbz): the dense level's extent
  int hh = 0, n2 = 0;        // ceil(pbz/2), 3*hh
  int umx = 0, umy = 0;      // nx/2+1, ny/2+1
  int psym = 0;              // 1 (even pbz): packed symmetric tiles of (S B)^{-1}, see precond
  int ntr = 0;               // tile rows per half, ceil(n2 / 16)
  double2 *binv64 = nullptr; // psym 0: [umy][umx][2][n2][n2] column-major inverse halves;
                             // psym 1: [umy][umx][2][ntr (ntr+1) / 2][256] packed tiles
  float2 *binv32 = nullptr;
  // circulant-plus-diagonal (opt.diag_steps > 0): Delta = 1/alpha_j - alpha~^{-1} per occupied
  // voxel [nocc]; two compact [R][3][nocc] work vectors for the fixed-point steps
  double2 *pdelta = nullptr;
  double2 *pdt = nullptr, *pdz = nullptr;

  // Krylov state (FP64)
  double2 *V = nullptr;      // [restart+1][R][3N]
  double2 *work = nullptr;   // [R][3N]  w / z scratch
  double2 *work2 = nullptr;  // [R][3N]
  double2 *bvec = nullptr;   // [R][3N] right-hand side
  double2 *xvec = nullptr;   // [R][3N] iterate
  double2 *H = nullptr;      // [R][restart+1][restart]
  double2 *givens = nullptr; // [R][restart][2] (c real in .x, s complex)
  double2 *gvec = nullptr;   // [R][restart+1]
  double2 *hcol = nullptr;   // [R][restart+1] projections
  double2 *hcol2 = nullptr;  // [R][restart+1]
  double2 *ycoef = nullptr;  // [R][restart+1]
  double2 *hnrm = nullptr;   // [R][kMaxM] squared norm after the projection
  double2 *hraw = nullptr;   // [R][2 kMaxM] raw projections and Gram overlaps of one iteration
  double2 *lmat = nullptr;   // [R][m+1][m+1] strictly lower triangle of the basis Gram matrix
  double *partial = nullptr; // reduction partials
  size_t partial_elems = 0;
  double *dscal = nullptr;   // [R][16] device scalars
  double *vsc = nullptr;     // [R][kMaxM] 1 / norm of each (unnormalised) basis vector
  double *hpin = nullptr;    // pinned host buffer [R][16]: a restart cycle's results
  double2 *stage = nullptr;  // [R][8] device staging of small per-RHS results for hpin
  int *hlive = nullptr;      // pinned host copy of the cycle's summary flag (read per segment)
  int *dflag = nullptr;      // device error flags [4]
  int *ctl = nullptr;        // device control of a GMRES cycle [1 + 4R] (krylov.hip)
  int *ones = nullptr;       // [R] ones: "every right-hand side" for the reductions
  double *bnrm = nullptr;    // [R] the norm each right-hand side's stopping test is relative to
  double *cres = nullptr;    // [3R] a cycle's results (squared residual norms, steps)
  double *hist = nullptr;    // [R][hist_cap] residual estimate after every GMRES step
  int hist_cap = 0;
  double2 *adj = nullptr;    // [3 nocc] forward solution kept across dda_grad_cext's two solves
  const int *act = nullptr;  // inside a GMRES cycle: the per-right-hand-side flags with which
                             // the cycle's operator and preconditioner launches skip the
                             // right-hand sides that have stopped; null elsewhere
  hipStream_t cap_st = nullptr;  // private stream on which restart cycles are captured
  struct CycleGraph {
    int nrhs, fp32;
    double tol;
    int maxit;
    const double2 *b;
    double2 *x;
    int part;  // -1 start of a cycle, k >= 0 its k-th segment of steps, -2 its end
    hipGraphExec_t exec;
  };
  std::vector<CycleGraph> graphs;  // captured restart cycles (invalid once the preconditioner
                                   // is rebuilt)
  double t_setup = 0.0, t_build = 0.0;  // seconds in dda_create / the last build

  dda::Profiler prof;
};

// ----------------------------------------------------------------------------- internal entry points

namespace dda {

// fft.hip — plain (setup) transforms on FP64 arrays, in place
void fft_rows_plain(dda_problem *p, const FftPlan &pl, double2 *data, long long rows, int inverse);
void fft_strided_plain(dda_problem *p, const FftPlan &pl, double2 *data, long long batch,
                       long long width, int inverse);

// operator.hip
// Validation, mean permittivity, occupied count and the compact index maps.
void operator_setup(dda_problem *p);
// Kernel spectra and z-pass tuning (after the work buffers exist).
void operator_spectrum_setup(dda_problem *p);
// Box [nrhs][3][N] <-> compact [nrhs][3][nocc]; to_box fills air from `fill` (or zeros).
void to_compact(dda_problem *p, int nrhs, const double2 *box, double2 *comp);
void to_box(dda_problem *p, int nrhs, const double2 *comp, const double2 *fill, double2 *box);
void copy_to_frame(dda_problem *p, const uint8_t *mask, const double2 *eps);
void setup_alpha(dda_problem *p, int nrhs, const double *S_host);
void setup_rhs(dda_problem *p, int nrhs, const double *dir, const double *pol, double2 *b,
               int conjugate);
// y = A (s x) on compact FP64 vectors (fp32: FP32 transforms inside).  xscale_dev: optional
// per-RHS input scale s_r = xscale_dev[r * kMaxM] (used for unnormalised Krylov vectors).
void apply_operator(dda_problem *p, int nrhs, const double2 *x, double2 *y, int fp32,
                    const double *xscale_dev);
void apply_imag_conv(dda_problem *p, int nrhs, const double2 *x, double2 *y);

// precond.hip
void precond_build(dda_problem *p, double s_bar);
void apply_precond(dda_problem *p, int nrhs, const double2 *x, double2 *y, int fp32,
                   const double *xscale_dev);
void precond_free(dda_problem *p);

// krylov.hip
void krylov_alloc(dda_problem *p);
// Pick the tile shapes of the four x / y passes of the operator (first = FP_OP_X_FWD) or of the
// 2-level preconditioner (FP_PC_X_FWD) in precision pi (0 FP64, 1 FP32) by timing `apply` (one
// application of that product on nrhs right-hand sides) with each candidate; cached per
// (device, grid, nrhs, precision) for the process.  DDA_FFT_TUNE=0 keeps the launch rules.
void fft_tile_autotune(dda_problem *p, int first, int pi, int nrhs, const std::function<void()> &apply);
// Solve A x = b for nrhs RHS (b, x compact [nrhs][3 nocc]; x holds the initial guess).
void gmres_solve(dda_problem *p, int nrhs, const double2 *b, double2 *x, int fp32, double tol,
                 int maxit, dda_stats *st);
// Full solve including refinement mode.
dda_status solve_system(dda_problem *p, int nrhs, const double2 *b, double2 *x, dda_stats *st);
// Destroy the captured restart cycles (their launches hold the preconditioner's buffers).
void drop_graphs(dda_problem *p);

// xsec.hip
void cross_sections(dda_problem *p, int nrhs, const double *dir, const double *pol,
                    const double2 *c, double *cext, double *cabs, double *csca);
void grad_kernel(dda_problem *p, const double2 *c, const double2 *lam, double S, double2 *grad);

// reductions (krylov.hip): per-RHS sums of n-length arrays
int reduce_blocks(long long n);

// xsec.hip: waves per call of dda_cross_sections_noalloc, and the one-time lookup (per device,
// with it current) of the device address of that call's static scratch array
constexpr int kNoallocMaxRhs = 16;
hipError_t noalloc_scratch_init(int dev);

}  // namespace dda
