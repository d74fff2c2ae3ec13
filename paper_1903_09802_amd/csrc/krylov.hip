// Restarted GMRES(m), right-preconditioned, FP64 Arnoldi, per-RHS Hessenberg / Givens
// updates on the device, and the mixed-precision mode in which each restart cycle is one step
// of iterative refinement (FP32 operator and preconditioner inside the cycle, FP64 residual at
// the restart).  The paper runs GMRES to 1e-5 (Sec. 4); restarts are the variant it recommends
// for memory (Sec. 4-5).
//
// Basis vectors are stored unnormalised: vsc[r][i] = 1 / ||v~_i|| scales them wherever they
// are used (projection coefficients, the operator's input prologue, the solution update),
// which saves one full pass per iteration.
//
// Orthogonalisation is modified Gram-Schmidt written with one reduction per iteration (the
// inverse compact WY form of Swirydowicz, Langou, Ananthan, Yang and Thomas): the MGS
// sequence of projections (I - v_j v_j^H) ... (I - v_0 v_0^H) equals I - V T V^H with
// T = (I + L)^{-1}, L the strictly lower triangle of V^H V.  One pass over the basis gives both
// a = V^H w and the new row of L (the overlaps of v_j with v_0 .. v_{j-1}); a forward
// substitution on the device gives the MGS coefficients c = T a; a second pass forms
// w - V c and ||w - V c||^2.  Two reads of the basis per iteration, MGS's rounding behaviour
// (loss of orthogonality of order eps * cond), no host decision inside an iteration.  All
// reductions are fixed-order (per-block partials, then one ordered pass), so results repeat
// bit for bit.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "common.h"

namespace dda {

// DDA_VERBOSE=1 in the environment prints one line per restart cycle / refinement to stderr.
static bool verbose() {
  static const int v = [] {
    const char *e = std::getenv("DDA_VERBOSE");
    return e && e[0] && e[0] != '0' ? 1 : 0;
  }();
  return v != 0;
}

constexpr int kRedThreads = 256;
constexpr int kCH = 8;             // vectors per multi-dot sweep
constexpr int kSlots = 2 * kMaxM;  // reduction slots per RHS: projections, then Gram overlaps

int reduce_blocks(long long n) {
  long long b = (n + 1023) / 1024;
  return (int)std::max<long long>(1, std::min<long long>(1024, b));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the block of NQ complex values per thread; results in sh[q] (all threads see them).
template <int NQ>
__device__ __forceinline__ void block_sum(double2 (&acc)[NQ], double2 *sh /* [4][NQ] */) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double re = wave_sum(acc[q].x), im = wave_sum(acc[q].y);
    if (lane == 0) sh[wv * NQ + q] = make_double2(re, im);
  }
  __syncthreads();
  if ((int)threadIdx.x < NQ) {
    double2 t = make_double2(0.0, 0.0);
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = cadd(t, sh[w * NQ + threadIdx.x]);
    sh[threadIdx.x] = t;
  }
  __syncthreads();
}

// One pass over basis blocks 0 .. j for every active RHS:
//   partial slot i (i <= j):          sum_n conj(v~_i[n]) w[n]
//   partial slot kMaxM + k (k < j):   sum_n conj(v~_k[n]) v~_j[n]
// at partial[(r * kSlots + slot) * B + block].
__global__ void __launch_bounds__(kRedThreads) k_gs_dots(const double2 *V, long long vs_r,
                                                         long long vs_j, int j, const double2 *w,
                                                         long long ws_r, long long n3,
                                                         const int *active, double2 *partial,
                                                         int B) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  __shared__ double2 sh[4 * 2 * kCH];
  const double2 *wr = w + r * ws_r;
  const double2 *Vr = V + r * vs_r;
  const double2 *vj = Vr + (long long)j * vs_j;
  for (int i0 = 0; i0 <= j; i0 += kCH) {
    double2 acc[2 * kCH];
#pragma unroll
    for (int q = 0; q < 2 * kCH; ++q) acc[q] = make_double2(0.0, 0.0);
    const bool gram = i0 < j;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
         n += (long long)gridDim.x * blockDim.x) {
      const double2 wv = wr[n];
      const double2 jv = gram ? vj[n] : make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < kCH; ++q) {
        if (i0 + q <= j) {
          const double2 v = Vr[(long long)(i0 + q) * vs_j + n];
          acc[q] = cadd(acc[q], cmulcj(v, wv));
          if (i0 + q < j) acc[kCH + q] = cadd(acc[kCH + q], cmulcj(v, jv));
        }
      }
    }
    block_sum<2 * kCH>(acc, sh);
    const int t = threadIdx.x;
    if (t < kCH && i0 + t <= j)
      partial[((long long)r * kSlots + i0 + t) * B + blockIdx.x] = sh[t];
    else if (t >= kCH && t < 2 * kCH && i0 + t - kCH < j)
      partial[((long long)r * kSlots + kMaxM + i0 + t - kCH) * B + blockIdx.x] = sh[t];
    __syncthreads();
  }
}

// Ordered sum of one partial row over its B blocks; the result is valid in thread 0.
__device__ __forceinline__ double2 ordered_sum(const double2 *row, int B, double2 *sh) {
  double2 acc = make_double2(0.0, 0.0);
  for (int b = threadIdx.x; b < B; b += blockDim.x) acc = cadd(acc, row[b]);
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] = cadd(sh[threadIdx.x], sh[threadIdx.x + s]);
    __syncthreads();
  }
  return sh[0];
}

// Reduce the 2j + 1 slots k_gs_dots wrote: out[r * kSlots + slot] (raw, unscaled sums).
__global__ void k_finalize_dots(const double2 *partial, int B, double2 *out, const int *active,
                                int j) {
  const int r = blockIdx.y, bx = blockIdx.x;
  if (!active[r]) return;
  const int slot = bx <= j ? bx : kMaxM + (bx - j - 1);
  __shared__ double2 sh[kRedThreads];
  const double2 v = ordered_sum(partial + ((long long)r * kSlots + slot) * B, B, sh);
  if (threadIdx.x == 0) out[r * kSlots + slot] = v;
}

// MGS coefficients from one reduction (one 64-lane block per RHS): store row j of
// L (L_jk = v_j^H v_k, k < j, with the basis scales applied), then c = (I + L)^{-1} a by
// forward substitution, a_i = v_i^H w, each step's dot product split over the lanes.  c goes
// to hcol (the Hessenberg column) and c_i * vsc_i to ycoef (the coefficients of the
// unnormalised basis in the update).
__global__ void __launch_bounds__(64) k_mgs_coef(int j, const double2 *raw, double2 *L, int lm,
                                                 const double *vsc, double2 *hcol, double2 *ycoef,
                                                 const int *active, int nrhs) {
  const int r = blockIdx.x, lane = threadIdx.x;
  if (r >= nrhs || !active[r]) return;
  __shared__ double2 c[kMaxM];
  const double *sr = vsc + r * kMaxM;
  double2 *Lr = L + (long long)r * lm * lm;  // [lm][lm], lm = restart + 1
  const double2 *rr = raw + r * kSlots;
  for (int k = lane; k < j; k += 64) Lr[j * lm + k] = cconj(cscale(rr[kMaxM + k], sr[k] * sr[j]));
  __syncthreads();
  for (int i = 0; i <= j; ++i) {
    double re = 0.0, im = 0.0;
    for (int k = lane; k < i; k += 64) {
      const double2 t = cmul(Lr[i * lm + k], c[k]);
      re += t.x;
      im += t.y;
    }
    re = wave_sum(re);
    im = wave_sum(im);
    if (lane == 0) {
      const double2 a = cscale(rr[i], sr[i]);
      const double2 ci = make_double2(a.x - re, a.y - im);
      c[i] = ci;
      hcol[r * kMaxM + i] = ci;
      ycoef[r * kMaxM + i] = cscale(ci, sr[i]);
    }
    __syncthreads();
  }
}

// out[r * kMaxM + i] = s_i * sum_b partial[(r * kSlots + i) * B + b] (ordered), and, if coef,
// coef[r * kMaxM + i] = s_i * out[...]; s_i = vsc[r * kMaxM + i] (1 when vsc is null).
// With islot >= 0 a single slot islot is reduced into out[r * kMaxM].
__global__ void k_finalize(const double2 *partial, int B, double2 *out, double2 *coef,
                           const double *vsc, const int *active, int islot) {
  const int i = islot >= 0 ? islot : blockIdx.x, r = blockIdx.y;
  const int io = islot >= 0 ? 0 : blockIdx.x;
  if (!active[r]) return;
  __shared__ double2 sh[kRedThreads];
  const double2 sum = ordered_sum(partial + ((long long)r * kSlots + i) * B, B, sh);
  if (threadIdx.x == 0) {
    const double s = vsc ? vsc[r * kMaxM + i] : 1.0;
    const double2 h = cscale(sum, s);
    out[r * kMaxM + io] = h;
    if (coef) coef[r * kMaxM + io] = cscale(h, s);
  }
}

// w -= sum_i V_i c_i (c = coef[r * kMaxM + i]); if nrm_partial: partial ||w||^2 (in .x)
__global__ void __launch_bounds__(kRedThreads) k_multiaxpy(const double2 *V, long long vs_r,
                                                           long long vs_j, int nvec,
                                                           const double2 *coef, double2 *w,
                                                           long long ws_r, long long n3,
                                                           const int *active,
                                                           double2 *nrm_partial, int B) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  __shared__ double2 c[kMaxM];
  __shared__ double2 sh[4];
  for (int i = threadIdx.x; i < nvec; i += blockDim.x) c[i] = coef[r * kMaxM + i];
  __syncthreads();
  double2 *wr = w + r * ws_r;
  const double2 *Vr = V + r * vs_r;
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    double2 v = wr[n];
#pragma unroll 8
    for (int i = 0; i < nvec; ++i) v = csub(v, cmul(Vr[i * vs_j + n], c[i]));
    wr[n] = v;
    acc[0].x += v.x * v.x + v.y * v.y;
  }
  if (!nrm_partial) return;
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) nrm_partial[((long long)r * kSlots) * B + blockIdx.x] = sh[0];
}

// out = sum_i V_i y_i  (y = coef[r * kMaxM + i], zero beyond a RHS's cut); with jcut, right-hand
// side r combines only its first jcut[r] vectors
__global__ void k_combine(const double2 *V, long long vs_r, long long vs_j, int nvec,
                          const double2 *coef, double2 *out, long long os_r, long long n3,
                          const int *jcut) {
  const int r = blockIdx.y;
  __shared__ double2 c[kMaxM];
  const int nv = jcut ? min(nvec, jcut[r]) : nvec;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) c[i] = coef[r * kMaxM + i];
  __syncthreads();
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    double2 v = make_double2(0.0, 0.0);
    for (int i = 0; i < nv; ++i) v = cadd(v, cmul(V[r * vs_r + i * vs_j + n], c[i]));
    out[r * os_r + n] = v;
  }
}

// out = a + s * b (per element), s = +1 or -1; optional partial ||out||^2
__global__ void __launch_bounds__(kRedThreads) k_axpby(const double2 *a, const double2 *b,
                                                       double s, double2 *out, long long n3,
                                                       long long st_r, const int *active,
                                                       double2 *nrm_partial, int B) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  __shared__ double2 sh[4];
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    const long long o = r * st_r + n;
    const double2 v = make_double2(a[o].x + s * b[o].x, a[o].y + s * b[o].y);
    out[o] = v;
    acc[0].x += v.x * v.x + v.y * v.y;
  }
  if (!nrm_partial) return;
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) nrm_partial[((long long)r * kSlots) * B + blockIdx.x] = sh[0];
}

// partial ||a||^2
__global__ void __launch_bounds__(kRedThreads) k_norm2(const double2 *a, long long n3,
                                                       long long st_r, double2 *nrm_partial,
                                                       int B) {
  const int r = blockIdx.y;
  __shared__ double2 sh[4];
  double2 acc[1] = {make_double2(0.0, 0.0)};
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    const double2 v = a[r * st_r + n];
    acc[0].x += v.x * v.x + v.y * v.y;
  }
  block_sum<1>(acc, sh);
  if (threadIdx.x == 0) nrm_partial[((long long)r * kSlots) * B + blockIdx.x] = sh[0];
}

// out[n] = in[n] * scal[r * sstride]
__global__ void k_scale(const double2 *in, double2 *out, long long n3, long long ins_r,
                        long long outs_r, const double *scal, int sstride, const int *active) {
  const int r = blockIdx.y;
  if (active && !active[r]) return;
  const double s = scal[r * sstride];
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    const double2 v = in[r * ins_r + n];
    out[r * outs_r + n] = make_double2(v.x * s, v.y * s);
  }
}

// ----------------------------------------------------------------------------- device control

// Every step's continue / stop decision is taken on the device, so a restart cycle runs without
// the host: the control block ctl (ints) holds
//   [0]                 live: some right-hand side is still iterating in this cycle; every
//                       kernel of the operator and the preconditioner launched inside the cycle
//                       returns at once when it is 0
//   [1, 1 + R)          active: right-hand side r takes further steps in this cycle
//   [1 + R, 1 + 2R)     jcut: steps r took in this cycle (the size of its least-squares problem)
//   [1 + 2R, 1 + 3R)    iters: steps r took in this solve
//   [1 + 3R, 1 + 4R)    want: r runs this cycle (set by the host between cycles)
// The host reads the results once per cycle (true residuals and step counts).
__host__ __device__ __forceinline__ int *ctl_active(int *c, int) { return c + 1; }
__host__ __device__ __forceinline__ int *ctl_jcut(int *c, int R) { return c + 1 + R; }
__host__ __device__ __forceinline__ int *ctl_iters(int *c, int R) { return c + 1 + 2 * R; }
__host__ __device__ __forceinline__ int *ctl_want(int *c, int R) { return c + 1 + 3 * R; }

// Start of a solve: no steps taken, nothing active.
__global__ void k_ctl_reset(int *ctl, int R) {
  for (int i = threadIdx.x; i < 1 + 4 * R; i += blockDim.x) ctl[i] = 0;
}

// Start of a cycle (basis vector 0 is the residual itself): active = want, g = (beta, 0, ...),
// vsc[0] = 1 / beta with beta = sqrt(rn2), live = any active.  One 64-lane block (nrhs <= 64).
__global__ void k_cycle_init(const double2 *rn2, double2 *g, int m, double *vsc, int *ctl, int R,
                             int nrhs) {
  const int r = threadIdx.x;
  bool on = false;
  if (r < nrhs) {
    on = ctl_want(ctl, R)[r] != 0;
    ctl_active(ctl, R)[r] = on ? 1 : 0;
    ctl_jcut(ctl, R)[r] = 0;
    if (on) {
      const double beta = sqrt(rn2[r * kMaxM].x);
      for (int i = 0; i <= m; ++i) g[r * (m + 1) + i] = make_double2(0.0, 0.0);
      g[r * (m + 1)] = make_double2(beta, 0.0);
      vsc[r * kMaxM] = beta > 0.0 ? 1.0 / beta : 0.0;
    }
  }
  const unsigned long long any = __ballot(on);
  if (threadIdx.x == 0) ctl[0] = any != 0ull ? 1 : 0;
}

// Column j of the Hessenberg matrix from the projections and ||w||^2, previous rotations, a
// new rotation, the updated residual estimate |g_{j+1}| (dscal[r*8]), ||w|| (dscal[r*8+2]) and
// the scale 1/||w|| of the new basis vector (vsc[r][j+1]); then the step's decision: the
// estimate relative to bnrm[r] is recorded in the history, and right-hand side r stops when it
// is at most tol, w vanished (breakdown), the estimate is not finite, the step cap is reached
// or the cycle is full.  live = some right-hand side continues.  One 64-lane block.
__global__ void k_arnoldi(int j, int m, double2 *H, double2 *giv, double2 *g, const double2 *h1,
                          const double2 *nrm2, double *dscal, double *vsc, int *ctl, int R,
                          int nrhs, const double *bnrm, double tol, int maxit, double *hist,
                          int hcap) {
  const int r = threadIdx.x;
  bool keep = false;
  int *active = ctl_active(ctl, R);
  if (r < nrhs && active[r]) {
    double2 *Hr = H + (long long)r * (m + 1) * m;
    double2 *gr = g + r * (m + 1);
    double2 *cs = giv + (long long)r * m * 2;
    for (int i = 0; i <= j; ++i) Hr[i * m + j] = h1[r * kMaxM + i];
    const double hn = sqrt(nrm2[r * kMaxM].x);
    Hr[(j + 1) * m + j] = make_double2(hn, 0.0);
    for (int i = 0; i < j; ++i) {
      const double c = cs[2 * i].x;
      const double2 s = cs[2 * i + 1];
      const double2 a = Hr[i * m + j], b = Hr[(i + 1) * m + j];
      const double2 t = cadd(cscale(a, c), cmul(s, b));
      Hr[(i + 1) * m + j] = csub(cscale(b, c), cmulcj(s, a));
      Hr[i * m + j] = t;
    }
    const double2 a = Hr[j * m + j], b = Hr[(j + 1) * m + j];
    const double aa = sqrt(a.x * a.x + a.y * a.y), bb = sqrt(b.x * b.x + b.y * b.y);
    const double den = sqrt(aa * aa + bb * bb);
    double c;
    double2 s;
    if (den == 0.0) { c = 1.0; s = make_double2(0.0, 0.0); }
    else if (aa == 0.0) { c = 0.0; s = make_double2(1.0, 0.0); }
    else {
      c = aa / den;
      const double2 ph = make_double2(a.x / aa, a.y / aa);
      s = cscale(cmul(ph, cconj(b)), 1.0 / den);
    }
    cs[2 * j] = make_double2(c, 0.0);
    cs[2 * j + 1] = s;
    Hr[j * m + j] = cadd(cscale(a, c), cmul(s, b));
    Hr[(j + 1) * m + j] = make_double2(0.0, 0.0);
    const double2 gj = gr[j];
    gr[j + 1] = make_double2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));  // -conj(s) g_j
    gr[j] = cscale(gj, c);
    const double2 e = gr[j + 1];
    const double en = sqrt(e.x * e.x + e.y * e.y);
    dscal[r * 8 + 0] = en;
    dscal[r * 8 + 2] = hn;
    if (j + 1 < kMaxM) vsc[r * kMaxM + j + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
    int *iters = ctl_iters(ctl, R);
    const int it = iters[r] + 1;
    iters[r] = it;
    const double est = bnrm[r] > 0.0 ? en / bnrm[r] : en;
    if (hist && it <= hcap) hist[(long long)r * hcap + it - 1] = est;
    if (est <= tol || hn == 0.0 || !isfinite(est) || it >= maxit || j == m - 1) {
      active[r] = 0;
      ctl_jcut(ctl, R)[r] = j + 1;
    } else {
      keep = true;
    }
  }
  const unsigned long long any = __ballot(keep);
  if (threadIdx.x == 0) ctl[0] = any != 0ull ? 1 : 0;
}

// y = H(0:jc, 0:jc)^{-1} g(0:jc) (upper triangular), zero beyond jc; stored as the
// combination coefficients y_i * vsc_i of the unnormalised basis.
__global__ void k_trisolve(const double2 *H, const double2 *g, int m, const int *jcut,
                           const double *vsc, double2 *y, int nrhs) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  const double2 *Hr = H + (long long)r * (m + 1) * m;
  const double2 *gr = g + r * (m + 1);
  const int jc = jcut[r];
  for (int i = 0; i < kMaxM; ++i) y[r * kMaxM + i] = make_double2(0.0, 0.0);
  for (int i = jc - 1; i >= 0; --i) {
    double2 acc = gr[i];
    for (int q = i + 1; q < jc; ++q) acc = csub(acc, cmul(Hr[i * m + q], y[r * kMaxM + q]));
    y[r * kMaxM + i] = cdiv(acc, Hr[i * m + i]);
  }
  for (int i = 0; i < jc; ++i) y[r * kMaxM + i] = cscale(y[r * kMaxM + i], vsc[r * kMaxM + i]);
}

// out[r] = sqrt(in[r * kMaxM].x)
__global__ void k_sqrt_slot(const double2 *in, double *out, int nrhs) {
  const int r = threadIdx.x;
  if (r < nrhs) out[r] = sqrt(in[r * kMaxM].x);
}

// The results the host reads after a cycle: res[r] = ||b - A x||^2, res[R + r] = the squared
// norm the stopping test uses (||P^{-1}(b - A x)||^2 when left preconditioned), res[2R + r] =
// steps taken.
__global__ void k_cycle_results(const double2 *tr2, const double2 *rr2, const int *ctl, int R,
                                int nrhs, double *res) {
  const int r = threadIdx.x;
  if (r >= nrhs) return;
  res[r] = tr2[r * kMaxM].x;
  res[R + r] = rr2[r * kMaxM].x;
  res[2 * R + r] = (double)ctl[1 + 2 * R + r];
}

// ----------------------------------------------------------------------------- host side

static inline dim3 grid_r(int B, int nrhs) { return dim3((unsigned)B, (unsigned)nrhs); }

struct Kry {
  dda_problem *p;
  int nrhs, B, m;
  long long n3;
  double2 *partial;
  int *d_active;
  int *d_jcut;
};

static void sync_active(dda_problem *p, int *d, const std::vector<int> &h) {
  HIPCHK(hipMemcpyAsync(d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, p->st));
}
// The same, skipped when the device copy `dev` already holds h (a copy from pageable memory can
// wait for the stream; the flags change only when a right-hand side stops).
static void sync_active_changed(dda_problem *p, int *d, const std::vector<int> &h,
                                std::vector<int> &dev) {
  if (h == dev) return;
  sync_active(p, d, h);
  dev = h;
}

static void finalize(Kry &K, int nvec, double2 *out, double2 *coef, const double *vsc,
                     int islot = -1) {
  hipLaunchKernelGGL(k_finalize, dim3(nvec, K.nrhs), dim3(kRedThreads), 0, K.p->st, K.partial, K.B,
                     out, coef, vsc, K.d_active, islot);
  HIPCHK(hipGetLastError());
}

// ||a_r||^2 into dst[r * kMaxM] (device), for every RHS
static void norm2_dev(Kry &K, const double2 *a, long long st_r, double2 *dst) {
  dda_problem *p = K.p;
  {
    KTimer t(&p->prof, p->st, "kry_norm", 16.0 * K.n3 * K.nrhs);
    hipLaunchKernelGGL(k_norm2, grid_r(K.B, K.nrhs), dim3(kRedThreads), 0, p->st, a, K.n3, st_r,
                       K.partial, K.B);
  }
  hipLaunchKernelGGL(k_finalize, dim3(1, K.nrhs), dim3(kRedThreads), 0, p->st, K.partial, K.B, dst,
                     nullptr, nullptr, p->ones, -1);
  HIPCHK(hipGetLastError());
}

// out[r * cnt + q] = in[r * stride + q] for r < nrhs, q < cnt: per-RHS slots made contiguous
__global__ void k_pack_slots(const double2 *in, long long stride, int cnt, int nrhs, double2 *out) {
  for (int e = threadIdx.x; e < cnt * nrhs; e += blockDim.x) {
    const int r = e / cnt, q = e - r * cnt;
    out[e] = in[r * stride + q];
  }
}

// cnt complex slots per right-hand side (stride apart on the device) to host[r * cnt + q]:
// packed on the device, then one plain copy into pinned memory
static void copy_slots(dda_problem *p, const double2 *src, long long stride, int cnt, int nrhs,
                       double2 *host) {
  hipLaunchKernelGGL(k_pack_slots, dim3(1), dim3(256), 0, p->st, src, stride, cnt, nrhs, p->stage);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(p->hpin, p->stage, sizeof(double2) * cnt * nrhs, hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  std::memcpy(host, p->hpin, sizeof(double2) * cnt * nrhs);
}

static void read_scalars(dda_problem *p, const double2 *src, int nrhs, std::vector<double> &out) {
  std::vector<double2> tmp(nrhs);
  copy_slots(p, src, kMaxM, 1, nrhs, tmp.data());
  out.resize(nrhs);
  for (int r = 0; r < nrhs; ++r) out[r] = tmp[r].x;
}

// One GMRES solve's fixed configuration: what a captured cycle depends on besides the handle.
struct GmresCfg {
  int nrhs, fp32, m, maxit;
  double tol;
  bool prec, left;
  long long vs_r, vs_j;
  const double2 *b;
  double2 *x;
};

// r = b - A x (FP64 operator) into basis block 0 with ||r||^2 in hcol2; left preconditioned,
// hnrm takes ||r||^2 and r becomes P^{-1} r with its squared norm in hcol2.  Then the results
// the host reads (k_cycle_results).  Every right-hand side takes part (active = 1 for all is
// not needed: the reductions here ignore the flags).
static void enqueue_residual(Kry &K, const GmresCfg &c) {
  dda_problem *p = K.p;
  const int nrhs = c.nrhs;
  double2 *rv = p->V;
  apply_operator(p, nrhs, c.x, p->work, 0, nullptr);
  {
    KTimer t(&p->prof, p->st, "kry_residual", 48.0 * K.n3 * nrhs);
    hipLaunchKernelGGL(k_axpby, grid_r(K.B, nrhs), dim3(kRedThreads), 0, p->st, c.b, p->work, -1.0,
                       rv, K.n3, K.n3, nullptr, K.partial, K.B);
  }
  hipLaunchKernelGGL(k_finalize, dim3(1, nrhs), dim3(kRedThreads), 0, p->st, K.partial, K.B,
                     c.left ? p->hnrm : p->hcol2, nullptr, nullptr, p->ones, -1);
  HIPCHK(hipGetLastError());
  if (c.left) {
    apply_precond(p, nrhs, rv, rv, p->prec_fp32, nullptr);
    {
      KTimer t(&p->prof, p->st, "kry_norm", 16.0 * K.n3 * nrhs);
      hipLaunchKernelGGL(k_norm2, grid_r(K.B, nrhs), dim3(kRedThreads), 0, p->st, rv, K.n3, K.n3,
                         K.partial, K.B);
    }
    hipLaunchKernelGGL(k_finalize, dim3(1, nrhs), dim3(kRedThreads), 0, p->st, K.partial, K.B,
                       p->hcol2, nullptr, nullptr, p->ones, -1);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(k_cycle_results, dim3(1), dim3(64), 0, p->st, c.left ? p->hnrm : p->hcol2,
                     p->hcol2, p->ctl, p->R, nrhs, p->cres);
  HIPCHK(hipGetLastError());
}

// A restart cycle runs in parts: its start, its steps in segments of growing length
// (steps [0, 4), [4, 12), [12, 28), [28, 60), ... up to m), and its end.  Between two segments
// the host reads one device flag (some right-hand side still iterating) and launches no more
// segments once it is 0, so a cycle that finishes early does not launch its remaining steps;
// within a segment, steps of stopped right-hand sides do no work.
static int segment_end(int j0, int m) { return std::min(m, j0 == 0 ? 4 : 2 * j0 + 4); }

// Part -1: start of the cycle for the right-hand sides the host marked in `want`.
// Part  k: the steps of segment k, each w = A P^{-1} v~_j (or P^{-1} A v~_j when left) into
//          basis block j + 1 with v~_j scaled by 1 / ||v~_j|| on the way in, MGS in one
//          reduction (a = V^H w and row j of L, c = (I + L)^{-1} a, w -= V c), and the device
//          decision of k_arnoldi.
// Part -2: the end: x += P^{-1}(V y) (x += V y when left) and the new residual.
static void enqueue_part(Kry &K, const GmresCfg &c, int part) {
  dda_problem *p = K.p;
  const int nrhs = c.nrhs, m = c.m;
  const long long n3 = K.n3, vs_r = c.vs_r, vs_j = c.vs_j;
  if (part == -1) {
    hipLaunchKernelGGL(k_cycle_init, dim3(1), dim3(64), 0, p->st, p->hcol2, p->gvec, m, p->vsc,
                       p->ctl, p->R, nrhs);
    HIPCHK(hipGetLastError());
    return;
  }
  if (part == -2) {
    hipLaunchKernelGGL(k_trisolve, dim3(1), dim3(64), 0, p->st, p->H, p->gvec, m, K.d_jcut, p->vsc,
                       p->ycoef, nrhs);
    {
      KTimer t(&p->prof, p->st, "kry_combine", 16.0 * n3 * (m + 1) * nrhs);
      hipLaunchKernelGGL(k_combine, grid_r(K.B, nrhs), dim3(kRedThreads), 0, p->st, p->V, vs_r,
                         vs_j, m, p->ycoef, p->work2, n3, n3, K.d_jcut);
    }
    HIPCHK(hipGetLastError());
    if (c.prec && !c.left) apply_precond(p, nrhs, p->work2, p->work2, c.fp32, nullptr);
    hipLaunchKernelGGL(k_axpby, grid_r(K.B, nrhs), dim3(kRedThreads), 0, p->st, c.x, p->work2, 1.0,
                       c.x, n3, n3, nullptr, nullptr, K.B);
    HIPCHK(hipGetLastError());
    enqueue_residual(K, c);
    return;
  }
  int j0 = 0;
  for (int k = 0; k < part; ++k) j0 = segment_end(j0, m);
  const int j1 = segment_end(j0, m);
  p->act = K.d_active;  // the products of a step skip the right-hand sides that have stopped
  try {
    for (int j = j0; j < j1; ++j) {
      double2 *vjj = p->V + (long long)j * vs_j;
      double2 *w = p->V + (long long)(j + 1) * vs_j;
      if (c.left) {
        apply_operator(p, nrhs, vjj, p->work2, c.fp32, p->vsc + j);
        apply_precond(p, nrhs, p->work2, w, c.fp32, nullptr);
      } else if (c.prec) {
        apply_precond(p, nrhs, vjj, p->work2, c.fp32, p->vsc + j);
        apply_operator(p, nrhs, p->work2, w, c.fp32, nullptr);
      } else {
        apply_operator(p, nrhs, vjj, w, c.fp32, p->vsc + j);
      }
      {
        KTimer t(&p->prof, p->st, "kry_gs_dots", 16.0 * n3 * (j + 2) * nrhs);
        hipLaunchKernelGGL(k_gs_dots, grid_r(K.B, nrhs), dim3(kRedThreads), 0, p->st, p->V, vs_r,
                           vs_j, j, w, vs_r, n3, K.d_active, K.partial, K.B);
      }
      hipLaunchKernelGGL(k_finalize_dots, dim3(2 * j + 1, nrhs), dim3(kRedThreads), 0, p->st,
                         K.partial, K.B, p->hraw, K.d_active, j);
      hipLaunchKernelGGL(k_mgs_coef, dim3(nrhs), dim3(64), 0, p->st, j, p->hraw, p->lmat, m + 1,
                         p->vsc, p->hcol, p->ycoef, K.d_active, nrhs);
      {
        KTimer t(&p->prof, p->st, "kry_multiaxpy", 16.0 * n3 * (j + 3) * nrhs);
        hipLaunchKernelGGL(k_multiaxpy, grid_r(K.B, nrhs), dim3(kRedThreads), 0, p->st, p->V, vs_r,
                           vs_j, j + 1, p->ycoef, w, vs_r, n3, K.d_active, K.partial, K.B);
      }
      finalize(K, 1, p->hnrm, nullptr, nullptr, 0);  // ||w - V c||^2 -> hnrm[r][0]
      hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(64), 0, p->st, j, m, p->H, p->givens, p->gvec,
                         p->hcol, p->hnrm, p->dscal, p->vsc, p->ctl, p->R, nrhs, p->bnrm, c.tol,
                         c.maxit, p->hist, p->hist_cap);
      HIPCHK(hipGetLastError());
    }
  } catch (...) {
    p->act = nullptr;
    throw;
  }
  p->act = nullptr;
}

// Enqueue one part: replay its HIP graph (captured on first use for this configuration), or
// launch its kernels one by one when graphs are off or per-kernel profiling is on.
static void launch_part(Kry &K, const GmresCfg &c, int part) {
  dda_problem *p = K.p;
  if (!p->opt.graph || p->prof.on) {
    enqueue_part(K, c, part);
    return;
  }
  hipGraphExec_t exec = nullptr;
  for (const auto &g : p->graphs)
    if (g.nrhs == c.nrhs && g.fp32 == c.fp32 && g.tol == c.tol && g.maxit == c.maxit &&
        g.b == c.b && g.x == c.x && g.part == part) {
      exec = g.exec;
      break;
    }
  if (!exec) {
    hipStream_t orig = p->st;
    HIPCHK(hipStreamBeginCapture(p->cap_st, hipStreamCaptureModeRelaxed));
    p->st = p->cap_st;
    hipGraph_t graph = nullptr;
    try {
      enqueue_part(K, c, part);
    } catch (...) {
      p->st = orig;
      if (hipStreamEndCapture(p->cap_st, &graph) == hipSuccess && graph) (void)hipGraphDestroy(graph);
      throw;
    }
    p->st = orig;
    HIPCHK(hipStreamEndCapture(p->cap_st, &graph));
    const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(e);
    p->graphs.push_back(dda_problem::CycleGraph{c.nrhs, c.fp32, c.tol, c.maxit, c.b, c.x, part, exec});
  }
  HIPCHK(hipGraphLaunch(exec, p->st));
}

// One restart cycle: start, segments until every right-hand side has stopped, end.  Nothing
// in a segment waits for the host; the host waits once per segment for the summary flag.
static void run_cycle(Kry &K, const GmresCfg &c) {
  dda_problem *p = K.p;
  launch_part(K, c, -1);
  for (int part = 0, j0 = 0; j0 < c.m; ++part) {
    launch_part(K, c, part);
    j0 = segment_end(j0, c.m);
    if (j0 >= c.m) break;
    HIPCHK(hipMemcpyAsync(p->hlive, p->ctl, sizeof(int), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    if (p->hlive[0] == 0) break;
  }
  launch_part(K, c, -2);
}

void drop_graphs(dda_problem *p) {
  for (auto &g : p->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
}

// Copy the cycle results to the host: true and test squared residual norms, steps per RHS.
static void read_results(dda_problem *p, int nrhs, std::vector<double> &tr2, std::vector<double> &rr2,
                         std::vector<int> &iters) {
  const int R = p->R;
  HIPCHK(hipMemcpyAsync(p->hpin, p->cres, sizeof(double) * 3 * R, hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  for (int r = 0; r < nrhs; ++r) {
    tr2[r] = p->hpin[r];
    rr2[r] = p->hpin[R + r];
    iters[r] = (int)p->hpin[2 * R + r];
  }
}

void gmres_solve(dda_problem *p, int nrhs, const double2 *b, double2 *x, int fp32, double tol,
                 int maxit, dda_stats *st) {
  const int m = p->opt.restart, R = p->R;
  const long long n3 = 3 * p->nocc;
  Kry K{p, nrhs, reduce_blocks(n3), m, n3, reinterpret_cast<double2 *>(p->partial),
        ctl_active(p->ctl, R), ctl_jcut(p->ctl, R)};
  GmresCfg c;
  c.nrhs = nrhs;
  c.fp32 = fp32;
  c.m = m;
  c.maxit = maxit;
  c.tol = tol;
  // Left preconditioning (the paper's P^{-1} A x = P^{-1} b): Krylov space of P^{-1} A, the
  // restart vector P^{-1}(b - A x), the update x += V y, and every test on the preconditioned
  // residual relative to ||P^{-1} b||.  Right preconditioning: A P^{-1}, x += P^{-1} V y, tests
  // on the true residual.  The preconditioner is applied in the precision it was built in.
  c.prec = p->opt.precond != 0;
  c.left = c.prec && p->opt.left_precond != 0;
  c.vs_r = n3;
  c.vs_j = (long long)R * n3;  // V is [m+1][R][n3]
  c.b = b;
  c.x = x;
  std::vector<int> act(nrhs, 1), incyc(nrhs, 0), iters(nrhs, 0), cycles(nrhs, 0), conv(nrhs, 0);
  std::vector<double> bt2, bn2, tr2(nrhs), rr2(nrhs), rel(nrhs, 0.0), trel(nrhs, 0.0);
  // ||b|| (and ||P^{-1} b||), the norms the tests are relative to, kept on the device too
  norm2_dev(K, b, n3, p->hcol2);
  if (c.left) {
    read_scalars(p, p->hcol2, nrhs, bt2);
    apply_precond(p, nrhs, b, p->work2, p->prec_fp32, nullptr);
    norm2_dev(K, p->work2, n3, p->hcol2);
  }
  hipLaunchKernelGGL(k_sqrt_slot, dim3(1), dim3(64), 0, p->st, p->hcol2, p->bnrm, nrhs);
  hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(256), 0, p->st, p->ctl, R);
  HIPCHK(hipGetLastError());
  read_scalars(p, p->hcol2, nrhs, bn2);
  if (!c.left) bt2 = bn2;
  // The restart residual b - A x is always formed with the FP64 operator: with fp32 != 0 every
  // restart is one step of iterative refinement (FP32 cycle, FP64 residual).
  auto take = [&]() {
    read_results(p, nrhs, tr2, rr2, iters);
    for (int r = 0; r < nrhs; ++r) {
      trel[r] = bt2[r] > 0 ? std::sqrt(tr2[r] / bt2[r]) : 0.0;
      rel[r] = bn2[r] > 0 ? std::sqrt(rr2[r] / bn2[r]) : 0.0;
      REQUIRE(std::isfinite(trel[r]) && std::isfinite(rel[r]), DDA_EDEVICE,
              "non-finite residual for right-hand side %d", r);
    }
  };
  enqueue_residual(K, c);
  take();
  for (int r = 0; r < nrhs; ++r)
    if (rel[r] <= tol || bn2[r] == 0.0) { act[r] = 0; conv[r] = 1; }
  int *want = ctl_want(p->ctl, R);
  while (true) {
    bool any = false;
    for (int r = 0; r < nrhs; ++r) {
      incyc[r] = act[r] && iters[r] < maxit;
      any = any || incyc[r];
      if (incyc[r]) cycles[r] += 1;
    }
    if (!any) break;
    HIPCHK(hipMemcpyAsync(want, incyc.data(), sizeof(int) * nrhs, hipMemcpyHostToDevice, p->st));
    run_cycle(K, c);
    take();
    if (verbose())
      for (int r = 0; r < nrhs; ++r)
        if (incyc[r])
          fprintf(stderr, "[dda] %s rhs %d cycle %d iters %d rel residual %.3e (true %.3e, tol %.1e)\n",
                  fp32 ? "fp32" : "fp64", r, cycles[r], iters[r], rel[r], trel[r], tol);
    for (int r = 0; r < nrhs; ++r) {
      if (!act[r]) continue;
      if (rel[r] <= tol) { act[r] = 0; conv[r] = 1; }
    }
  }
  // per-step residual estimates of every right-hand side whose stats ask for them
  for (int r = 0; r < nrhs; ++r) {
    if (!st[r].history || st[r].history_cap <= 0) continue;
    const int n = std::min({iters[r], st[r].history_cap, p->hist_cap});
    if (n > 0)
      HIPCHK(hipMemcpyAsync(st[r].history, p->hist + (long long)r * p->hist_cap, sizeof(double) * n,
                            hipMemcpyDeviceToHost, p->st));
    st[r].history_len = n;
  }
  HIPCHK(hipStreamSynchronize(p->st));
  for (int r = 0; r < nrhs; ++r) {
    st[r].iters += iters[r];
    st[r].cycles += cycles[r];
    st[r].rel_residual = trel[r];
    st[r].converged = conv[r];
  }
}

// ----------------------------------------------------------------------------- BiCGStab

// BiCGStab (the paper's second solver, Sec. 4), right-preconditioned, van der Vorst's
// recurrence with conjugated inner products.  Per-RHS scalars live on the device in
// bc[r * kMaxM + q]: q = 0 alpha, 1 omega, 2 beta, 3 rho, 4 breakdown flag; the dot products
// come reduced into hraw[r * kSlots + slot].  After a breakdown (a zero denominator) the
// rest of the iteration runs with alpha = omega = 0, which leaves x and r unchanged.

// partial slots 0, 1: sum conj(a_q) b_q over n for q < nq (b1 may equal a1 for a norm)
__global__ void __launch_bounds__(kRedThreads) k_dots2(const double2 *a0, const double2 *b0,
                                                       const double2 *a1, const double2 *b1,
                                                       int nq, long long n3, const int *active,
                                                       double2 *partial, int B) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  __shared__ double2 sh[4 * 2];
  double2 acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  const long long o = (long long)r * n3;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    acc[0] = cadd(acc[0], cmulcj(a0[o + n], b0[o + n]));
    if (nq > 1) acc[1] = cadd(acc[1], cmulcj(a1[o + n], b1[o + n]));
  }
  block_sum<2>(acc, sh);
  if ((int)threadIdx.x < nq) partial[((long long)r * kSlots + threadIdx.x) * B + blockIdx.x] = sh[threadIdx.x];
}

// Reduce slots [0, nq) into hraw[r * kSlots + slot].
__global__ void k_finalize_n(const double2 *partial, int B, double2 *out, const int *active) {
  const int r = blockIdx.y, slot = blockIdx.x;
  if (!active[r]) return;
  __shared__ double2 sh[kRedThreads];
  const double2 v = ordered_sum(partial + ((long long)r * kSlots + slot) * B, B, sh);
  if (threadIdx.x == 0) out[r * kSlots + slot] = v;
}

// Scalar updates, one thread per RHS.  stage 0: beta from rho_new = (rhat, r) (hraw slot 1);
// stage 1: alpha = rho / (rhat, v) (slot 0); stage 2: omega = (t, s) / (t, t) (slots 0, 1).
__global__ void k_bcg_scalars(int stage, const double2 *hraw, double2 *bc, const int *active,
                              int nrhs) {
  const int r = threadIdx.x;
  if (r >= nrhs || !active[r]) return;
  double2 *c = bc + r * kMaxM;
  const double2 *h = hraw + r * kSlots;
  const double2 zero = make_double2(0.0, 0.0);
  if (stage > 0 && c[4].x != 0.0) {  // broken down earlier in this iteration
    c[stage == 1 ? 0 : 1] = zero;
    return;
  }
  if (stage == 0) {
    const double2 rho_new = h[1];
    if (rho_new.x == 0.0 && rho_new.y == 0.0) {
      c[4] = make_double2(1.0, 0.0);
      c[2] = zero;
      return;
    }
    c[2] = cmul(cdiv(rho_new, c[3]), cdiv(c[0], c[1]));
    c[3] = rho_new;
  } else if (stage == 1) {
    const double2 den = h[0];
    if (den.x == 0.0 && den.y == 0.0) {
      c[4] = make_double2(1.0, 0.0);
      c[0] = zero;
      return;
    }
    c[0] = cdiv(c[3], den);
  } else {
    const double2 ts = h[0], tt = h[1];
    c[1] = (tt.x == 0.0 && tt.y == 0.0) ? zero : cdiv(ts, tt);
  }
}

// p = r + beta (p - omega v)
__global__ void k_bcg_p(const double2 *rr, double2 *pp, const double2 *v, const double2 *bc,
                        long long n3, const int *active) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  const double2 beta = bc[r * kMaxM + 2], omega = bc[r * kMaxM + 1];
  const long long o = (long long)r * n3;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x)
    pp[o + n] = cadd(rr[o + n], cmul(beta, csub(pp[o + n], cmul(omega, v[o + n]))));
}

// s = r - alpha v
__global__ void k_bcg_s(const double2 *rr, const double2 *v, double2 *s, const double2 *bc,
                        long long n3, const int *active) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  const double2 alpha = bc[r * kMaxM + 0];
  const long long o = (long long)r * n3;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x)
    s[o + n] = csub(rr[o + n], cmul(alpha, v[o + n]));
}

// x += alpha ph + omega sh; r = s - omega t; partial slot 0: ||r||^2, slot 1: (rhat, r)
__global__ void __launch_bounds__(kRedThreads) k_bcg_xr(double2 *x, const double2 *ph,
                                                        const double2 *shv, const double2 *s,
                                                        const double2 *t, double2 *rr,
                                                        const double2 *rh, const double2 *bc,
                                                        long long n3, const int *active,
                                                        double2 *partial, int B) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  __shared__ double2 sh[4 * 2];
  const double2 alpha = bc[r * kMaxM + 0], omega = bc[r * kMaxM + 1];
  const long long o = (long long)r * n3;
  double2 acc[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    x[o + n] = cadd(x[o + n], cadd(cmul(alpha, ph[o + n]), cmul(omega, shv[o + n])));
    const double2 rn = csub(s[o + n], cmul(omega, t[o + n]));
    rr[o + n] = rn;
    acc[0].x += rn.x * rn.x + rn.y * rn.y;
    acc[1] = cadd(acc[1], cmulcj(rh[o + n], rn));
  }
  block_sum<2>(acc, sh);
  if ((int)threadIdx.x < 2) partial[((long long)r * kSlots + threadIdx.x) * B + blockIdx.x] = sh[threadIdx.x];
}

// Start of a BiCGStab run: rhat = r, p = v = 0, alpha = omega = rho = 1, hraw slot 1 = ||r||^2
// (= (rhat, r)), breakdown flag cleared.
__global__ void k_bcg_init(const double2 *rr, double2 *rh, double2 *pp, double2 *v, long long n3,
                           const int *active) {
  const int r = blockIdx.y;
  if (!active[r]) return;
  const long long o = (long long)r * n3;
  for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < n3;
       n += (long long)gridDim.x * blockDim.x) {
    rh[o + n] = rr[o + n];
    pp[o + n] = make_double2(0.0, 0.0);
    v[o + n] = make_double2(0.0, 0.0);
  }
}

__global__ void k_bcg_init_scalars(double2 *hraw, double2 *bc, const int *active, int nrhs) {
  const int r = threadIdx.x;
  if (r >= nrhs || !active[r]) return;
  hraw[r * kSlots + 1] = hraw[r * kSlots + 0];
  double2 *c = bc + r * kMaxM;
  c[0] = c[1] = c[3] = make_double2(1.0, 0.0);
  c[2] = make_double2(0.0, 0.0);
  c[4] = make_double2(0.0, 0.0);
}

void bicgstab_solve(dda_problem *p, int nrhs, const double2 *b, double2 *x, double tol, int maxit,
                    dda_stats *st) {
  const long long n3 = 3 * p->nocc;
  REQUIRE(p->opt.restart >= 7, DDA_EINVAL, "BiCGStab needs restart >= 7 (work vectors)");
  Kry K{p, nrhs, reduce_blocks(n3), p->opt.restart, n3, reinterpret_cast<double2 *>(p->partial),
        ctl_active(p->ctl, p->R), ctl_jcut(p->ctl, p->R)};
  const bool prec = p->opt.precond != 0;
  const long long blk = (long long)p->R * n3;  // one basis block holds [R][n3]
  double2 *rr = p->V, *rh = p->V + blk, *pp = p->V + 2 * blk, *v = p->V + 3 * blk;
  double2 *s = p->V + 4 * blk, *t = p->V + 5 * blk, *ph = p->V + 6 * blk, *shv = p->V + 7 * blk;
  double2 *bc = p->ycoef;  // [R][kMaxM] complex: the first 5 per RHS hold the scalars
  const dim3 grid = grid_r(K.B, nrhs);
  std::vector<int> all(nrhs, 1), act(nrhs, 0), conv(nrhs, 0), iters(nrhs, 0), runs(nrhs, 0);
  std::vector<int> stuck(nrhs, 0);  // a run broke down before its first step: give up
  std::vector<double> bn2, rn2, rel(nrhs, 0.0);
  sync_active(p, K.d_active, all);
  norm2_dev(K, b, n3, p->hcol2);
  read_scalars(p, p->hcol2, nrhs, bn2);
  std::vector<double2> hb((size_t)nrhs), cb((size_t)nrhs * 5);  // ||r||^2 and the 5 scalars
  while (true) {
    // true residual r = b - A x for every RHS (FP64)
    sync_active(p, K.d_active, all);
    apply_operator(p, nrhs, x, p->work, 0, nullptr);
    {
      KTimer tm(&p->prof, p->st, "kry_residual", 48.0 * n3 * nrhs);
      hipLaunchKernelGGL(k_axpby, grid, dim3(kRedThreads), 0, p->st, b, p->work, -1.0, rr, n3, n3,
                         nullptr, K.partial, K.B);
    }
    finalize(K, 1, p->hcol2, nullptr, nullptr);
    read_scalars(p, p->hcol2, nrhs, rn2);
    bool any = false;
    for (int r = 0; r < nrhs; ++r) {
      rel[r] = bn2[r] > 0 ? std::sqrt(rn2[r] / bn2[r]) : 0.0;
      REQUIRE(std::isfinite(rel[r]), DDA_EDEVICE, "non-finite residual for right-hand side %d", r);
      conv[r] = rel[r] <= tol || bn2[r] == 0.0;
      act[r] = !conv[r] && iters[r] < maxit && !stuck[r];
      if (act[r]) { ++runs[r]; any = true; }
    }
    if (verbose())
      for (int r = 0; r < nrhs; ++r)
        fprintf(stderr, "[dda] bicgstab rhs %d run %d iters %d true rel residual %.3e (tol %.1e)\n",
                r, runs[r], iters[r], rel[r], tol);
    if (!any) break;
    sync_active(p, K.d_active, act);
    std::vector<int> dev_act = act;  // the flags on the device
    // hraw slot 0 = ||r||^2 for the active RHS, then rhat = r, p = v = 0, scalars
    {
      KTimer tm(&p->prof, p->st, "kry_norm", 16.0 * n3 * nrhs);
      hipLaunchKernelGGL(k_dots2, grid, dim3(kRedThreads), 0, p->st, rr, rr, rr, rr, 1, n3,
                         K.d_active, K.partial, K.B);
    }
    hipLaunchKernelGGL(k_finalize_n, dim3(1, nrhs), dim3(kRedThreads), 0, p->st, K.partial, K.B,
                       p->hraw, K.d_active);
    hipLaunchKernelGGL(k_bcg_init, grid, dim3(kRedThreads), 0, p->st, rr, rh, pp, v, n3, K.d_active);
    hipLaunchKernelGGL(k_bcg_init_scalars, dim3(1), dim3(64), 0, p->st, p->hraw, bc, K.d_active, nrhs);
    HIPCHK(hipGetLastError());
    const std::vector<int> run_start(iters), in_run(act);
    while (true) {
      bool left = false;
      for (int r = 0; r < nrhs; ++r) left = left || act[r];
      if (!left) break;
      hipLaunchKernelGGL(k_bcg_scalars, dim3(1), dim3(64), 0, p->st, 0, p->hraw, bc, K.d_active, nrhs);
      {
        KTimer tm(&p->prof, p->st, "bcg_p", 16.0 * n3 * 4 * nrhs);
        hipLaunchKernelGGL(k_bcg_p, grid, dim3(kRedThreads), 0, p->st, rr, pp, v, bc, n3, K.d_active);
      }
      if (prec) {
        apply_precond(p, nrhs, pp, ph, 0, nullptr);
        apply_operator(p, nrhs, ph, v, 0, nullptr);
      } else {
        apply_operator(p, nrhs, pp, v, 0, nullptr);
      }
      {
        KTimer tm(&p->prof, p->st, "bcg_dots", 16.0 * n3 * 2 * nrhs);
        hipLaunchKernelGGL(k_dots2, grid, dim3(kRedThreads), 0, p->st, rh, v, rh, v, 1, n3,
                           K.d_active, K.partial, K.B);
      }
      hipLaunchKernelGGL(k_finalize_n, dim3(1, nrhs), dim3(kRedThreads), 0, p->st, K.partial, K.B,
                         p->hraw, K.d_active);
      hipLaunchKernelGGL(k_bcg_scalars, dim3(1), dim3(64), 0, p->st, 1, p->hraw, bc, K.d_active, nrhs);
      {
        KTimer tm(&p->prof, p->st, "bcg_s", 16.0 * n3 * 3 * nrhs);
        hipLaunchKernelGGL(k_bcg_s, grid, dim3(kRedThreads), 0, p->st, rr, v, s, bc, n3, K.d_active);
      }
      if (prec) {
        apply_precond(p, nrhs, s, shv, 0, nullptr);
        apply_operator(p, nrhs, shv, t, 0, nullptr);
      } else {
        apply_operator(p, nrhs, s, t, 0, nullptr);
      }
      {
        KTimer tm(&p->prof, p->st, "bcg_dots", 16.0 * n3 * 2 * nrhs);
        hipLaunchKernelGGL(k_dots2, grid, dim3(kRedThreads), 0, p->st, t, s, t, t, 2, n3,
                           K.d_active, K.partial, K.B);
      }
      hipLaunchKernelGGL(k_finalize_n, dim3(2, nrhs), dim3(kRedThreads), 0, p->st, K.partial, K.B,
                         p->hraw, K.d_active);
      hipLaunchKernelGGL(k_bcg_scalars, dim3(1), dim3(64), 0, p->st, 2, p->hraw, bc, K.d_active, nrhs);
      {
        KTimer tm(&p->prof, p->st, "bcg_xr", 16.0 * n3 * 8 * nrhs);
        hipLaunchKernelGGL(k_bcg_xr, grid, dim3(kRedThreads), 0, p->st, x, prec ? ph : pp,
                           prec ? shv : s, s, t, rr, rh, bc, n3, K.d_active, K.partial, K.B);
      }
      hipLaunchKernelGGL(k_finalize_n, dim3(2, nrhs), dim3(kRedThreads), 0, p->st, K.partial, K.B,
                         p->hraw, K.d_active);
      HIPCHK(hipGetLastError());
      copy_slots(p, p->hraw, kSlots, 1, nrhs, hb.data());
      copy_slots(p, bc, kMaxM, 5, nrhs, cb.data());
      for (int r = 0; r < nrhs; ++r) {
        if (!act[r]) continue;
        // a breakdown left x and r unchanged: it ends the run and is not counted as a step
        const bool brk = cb[r * 5 + 4].x != 0.0;
        if (brk) {
          act[r] = 0;
          continue;
        }
        iters[r] += 1;
        const double est = bn2[r] > 0 ? std::sqrt(hb[r].x / bn2[r]) : 0.0;
        REQUIRE(std::isfinite(est), DDA_EDEVICE, "non-finite residual estimate (RHS %d)", r);
        if (st[r].history && iters[r] <= st[r].history_cap) {
          st[r].history[iters[r] - 1] = est;
          st[r].history_len = iters[r];
        }
        const double2 om = cb[r * 5 + 1];
        // stop this run at the updated tolerance, omega = 0 or the cap
        if (est <= tol || (om.x == 0.0 && om.y == 0.0) || iters[r] >= maxit) act[r] = 0;
      }
      sync_active_changed(p, K.d_active, act, dev_act);
    }
    for (int r = 0; r < nrhs; ++r)
      if (in_run[r] && iters[r] == run_start[r]) stuck[r] = 1;
  }
  for (int r = 0; r < nrhs; ++r) {
    st[r].iters += iters[r];
    st[r].cycles += runs[r];
    st[r].rel_residual = rel[r];
    st[r].converged = conv[r];
  }
}

dda_status solve_system(dda_problem *p, int nrhs, const double2 *b, double2 *x, dda_stats *st) {
  // counters start at zero; the caller's history buffers (in fields) are kept
  for (int r = 0; r < nrhs; ++r) {
    st[r].iters = st[r].cycles = st[r].refinements = st[r].converged = 0;
    st[r].rel_residual = 0.0;
    st[r].history_len = 0;
  }
  // precision 1: each GMRES(m) cycle applies the operator and the preconditioner in FP32 to an
  // FP64 basis, and each restart recomputes b - A x in FP64 (one refinement step per cycle)
  const int fp32 = p->opt.precision == 1 ? 1 : 0;
  if (p->opt.solver == 1)
    bicgstab_solve(p, nrhs, b, x, p->opt.tol, p->opt.max_iter, st);
  else
    gmres_solve(p, nrhs, b, x, fp32, p->opt.tol, p->opt.max_iter, st);
  if (fp32)
    for (int r = 0; r < nrhs; ++r) st[r].refinements = st[r].cycles;
  bool ok = true;
  for (int r = 0; r < nrhs; ++r) ok = ok && st[r].converged;
  return ok ? DDA_OK : DDA_NOT_CONVERGED;
}

__global__ void k_fill_int(int *a, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = v;
}

void krylov_alloc(dda_problem *p) {
  const int m = p->opt.restart;
  const int R = p->R;
  const long long n3 = 3 * p->nocc;
  {  // the basis and the work vectors, compact (3 N_occ entries per wave)
    const double need = 16.0 * n3 * ((double)R * (m + 1) + 4.0 * R + 1.0);
    size_t freeb = 0, totb = 0;
    HIPCHK(hipMemGetInfo(&freeb, &totb));
    REQUIRE(need < 0.9 * (double)freeb, DDA_ENOMEM,
            "Krylov basis of %d + 1 vectors x %d waves needs about %.2f GB, %.2f GB free", m, R,
            need / 1e9, freeb / 1e9);
  }
  HIPCHK(hipMalloc(&p->V, sizeof(double2) * (size_t)R * (m + 1) * n3));
  HIPCHK(hipMemsetAsync(p->V, 0, sizeof(double2) * (size_t)R * (m + 1) * n3, p->st));
  HIPCHK(hipMalloc(&p->work, sizeof(double2) * (size_t)R * n3));
  HIPCHK(hipMalloc(&p->work2, sizeof(double2) * (size_t)R * n3));
  HIPCHK(hipMalloc(&p->bvec, sizeof(double2) * (size_t)R * n3));
  HIPCHK(hipMalloc(&p->xvec, sizeof(double2) * (size_t)R * n3));
  HIPCHK(hipMalloc(&p->adj, sizeof(double2) * (size_t)n3));
  HIPCHK(hipMalloc(&p->H, sizeof(double2) * (size_t)R * (m + 1) * m));
  HIPCHK(hipMalloc(&p->givens, sizeof(double2) * (size_t)R * m * 2));
  HIPCHK(hipMalloc(&p->gvec, sizeof(double2) * (size_t)R * (m + 1)));
  HIPCHK(hipMalloc(&p->hcol, sizeof(double2) * (size_t)R * kMaxM));
  HIPCHK(hipMalloc(&p->hcol2, sizeof(double2) * (size_t)R * kMaxM));
  HIPCHK(hipMalloc(&p->ycoef, sizeof(double2) * (size_t)R * kMaxM));
  HIPCHK(hipMalloc(&p->hnrm, sizeof(double2) * (size_t)R * kMaxM));
  HIPCHK(hipMalloc(&p->hraw, sizeof(double2) * (size_t)R * kSlots));
  HIPCHK(hipMalloc(&p->lmat, sizeof(double2) * (size_t)R * (m + 1) * (m + 1)));
  const int B = reduce_blocks(n3);
  p->partial_elems = std::max<size_t>((size_t)R * kSlots * B * 2, (size_t)R * 512 * 4);
  HIPCHK(hipMalloc(&p->partial, sizeof(double) * p->partial_elems));
  HIPCHK(hipMalloc(&p->dscal, sizeof(double) * 16 * R));
  HIPCHK(hipMemset(p->dscal, 0, sizeof(double) * 16 * R));
  HIPCHK(hipHostMalloc(&p->hpin, sizeof(double) * 16 * R, hipHostMallocDefault));
  HIPCHK(hipHostMalloc(&p->hlive, sizeof(int) * 16, hipHostMallocDefault));
  HIPCHK(hipMalloc(&p->stage, sizeof(double2) * 8 * R));
  HIPCHK(hipMalloc(&p->vsc, sizeof(double) * kMaxM * R));
  HIPCHK(hipMemset(p->vsc, 0, sizeof(double) * kMaxM * R));
  HIPCHK(hipMalloc(&p->dflag, sizeof(int) * 4));
  HIPCHK(hipMemset(p->dflag, 0, sizeof(int) * 4));
  HIPCHK(hipMalloc(&p->ctl, sizeof(int) * (1 + 4 * R)));
  HIPCHK(hipMemset(p->ctl, 0, sizeof(int) * (1 + 4 * R)));
  HIPCHK(hipMalloc(&p->ones, sizeof(int) * R));
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, p->st, p->ones, R, 1);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMalloc(&p->bnrm, sizeof(double) * R));
  HIPCHK(hipMalloc(&p->cres, sizeof(double) * 3 * R));
  // per-step residual history of the GMRES solves, up to the step cap (at most 2^16 steps)
  p->hist_cap = std::min(p->opt.max_iter, 1 << 16);
  HIPCHK(hipMalloc(&p->hist, sizeof(double) * (size_t)R * p->hist_cap));
  HIPCHK(hipStreamCreateWithFlags(&p->cap_st, hipStreamNonBlocking));
}

}  // namespace dda
