// The 2-level circulant preconditioner (Sec. 3, 3.1): setup and application.
//
// The dense (z) level spans the occupied layers [pz0, pz0 + pbz) of the box, as the paper's
// box is the smallest one around the body; below, nz stands for that extent pbz.  Layers
// outside it hold only air, which M P^{-1} M never reads or keeps.
//
// Setup.  eq. Chan along x then y on the signed-offset kernel K(p, q, s) = d^3 G(p d,
// q d, s d) gives the generator c2_ab(pbar, qbar, s) (pbar < nx, qbar < ny, |s| < nz);
// its 2-D DFT over (pbar, qbar) gives lambda_ab(wx, wy, s).  For every Fourier mode the
// preconditioner is the dense 3nz x 3nz matrix
//     B(w)[(a, iz), (b, jz)] = alpha~^{-1} delta - lambda_ab(w, iz - jz)
// (Toeplitz along z).  Exact symmetries reduce the work:
//   * B(-wx, wy) = Sx B(wx, wy) Sx and B(wx, -wy) = Sy B Sy, Sx = diag(-1, 1, 1) per
//     component (the x / y parities of the six kernel blocks), so only modes with
//     0 <= wx <= nx/2, 0 <= wy <= ny/2 are inverted;
//   * B commutes with the z reflection (a, iz) -> s_a (a, nz-1-iz), s = (1, 1, -1), so
//     each B splits into an even and an odd half of size 3 ceil(nz/2) (a padding entry is
//     set to the identity when nz is odd).
// The halves are inverted explicitly (Gauss-Jordan with partial pivoting, blocked).  For
// even nz, S B_sigma is complex symmetric (S = diag(1, 1, -1) per component: the kernel
// blocks are symmetric in (a, b) up to the x / y parities, and the z reflection maps xz and
// yz onto their negatives), so its inverse Y = B_sigma^{-1} S is symmetric and only its lower
// triangle is stored, as 16 x 16 tiles; the application is B_sigma^{-1} v = Y (S v), a dense
// product of Y with the 8 complex columns of a mode (its up to 4 sign copies x 2 right-hand
// sides), run on the matrix cores.  For odd nz the middle z plane breaks that symmetry and
// the full halves are stored column-major.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>

#include "fft_kernels.h"

namespace dda {

// Some right-hand side of r0 .. r0 + nr - 1 is still iterating (act null: all are).
__device__ __forceinline__ bool rhs_any_on(const int *act, int r0, int nr) {
  if (!act) return true;
  for (int r = r0; r < r0 + nr; ++r)
    if (act[r]) return true;
  return false;
}

__device__ __forceinline__ void green6_chan(double x, double y, double z, double k, double d3,
                                            double w, double2 acc[6]) {
  const double r2 = x * x + y * y + z * z;
  if (r2 == 0.0 || w == 0.0) return;
  const double r = sqrt(r2);
  const double ir = 1.0 / r;
  const double h[3] = {x * ir, y * ir, z * ir};
  double sn, cs;
  sincos(k * r, &sn, &cs);
  const double2 e = make_double2(cs * ir * d3 * w, sn * ir * d3 * w);
  const double k2 = k * k, ir2 = ir * ir, kr = k * r;
  int c = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      const double P = h[a] * h[b];
      const double dl = (a == b) ? 1.0 : 0.0;
      acc[c] = cadd(acc[c], cmul(e, make_double2(k2 * (dl - P) - (dl - 3.0 * P) * ir2,
                                                 kr * (dl - 3.0 * P) * ir2)));
      ++c;
    }
}

// gen[c][s + nz - 1][qbar][pbar] = sum over p in {pbar, pbar - nx}, q in {qbar, qbar - ny} of
// wx(p) wy(q) K_c(p, q, s), with wx(pbar) = (nx - pbar)/nx, wx(pbar - nx) = pbar/nx (eq. Chan).
__global__ void k_chan_gen(double2 *gen, int nx, int ny, int nz, double k, double d) {
  const long long S = 2LL * nz - 1;
  const long long tot = S * ny * nx;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int pb = (int)(idx % nx);
  const int qb = (int)((idx / nx) % ny);
  const int si = (int)(idx / ((long long)nx * ny));
  const int s = si - (nz - 1);
  double2 acc[6];
  for (int c = 0; c < 6; ++c) acc[c] = make_double2(0.0, 0.0);
  const double d3 = d * d * d;
  const int ps[2] = {pb, pb - nx};
  const double wxs[2] = {(double)(nx - pb) / nx, (double)pb / nx};
  const int qs[2] = {qb, qb - ny};
  const double wys[2] = {(double)(ny - qb) / ny, (double)qb / ny};
  for (int u = 0; u < 2; ++u)
    for (int v = 0; v < 2; ++v) {
      const double w = wxs[u] * wys[v];
      if (w == 0.0) continue;
      green6_chan(ps[u] * d, qs[v] * d, s * d, k, d3, w, acc);
    }
  for (int c = 0; c < 6; ++c) gen[c * tot + idx] = acc[c];
}

// Assemble the transposed half-blocks X = B_sigma^T (row-major) for matrices
// [m0, m0 + count) of the list (mode u = m / 2, half = m % 2: 0 even, 1 odd).
// With sym != 0 the block written is M = S B_sigma (symmetric) instead of B_sigma^T.
template <typename TO>
__global__ void k_assemble(const double2 *lam, TO *out, long long m0, int nx, int ny,
                           int nz, int umx, int hh, int n2, double2 ati, int sym) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double2 *L = reinterpret_cast<double2 *>(smem_raw);  // [6][2nz-1]
  const long long m = m0 + blockIdx.x;
  const long long u = m / 2;
  const int half = (int)(m % 2);
  const int uy = (int)(u / umx), ux = (int)(u % umx);
  const long long S = 2LL * nz - 1;
  const long long plane = (long long)nx * ny;
  for (int e = threadIdx.x; e < 6 * S; e += blockDim.x) {
    const int c = e / (int)S;
    const int s = e - c * (int)S;
    L[e] = lam[((long long)c * S + s) * plane + (long long)uy * nx + ux];
  }
  __syncthreads();
  const double sig = half == 0 ? 1.0 : -1.0;
  const int h = nz / 2;
  TO *X = out + (long long)blockIdx.x * n2 * n2;
  for (long long e = threadIdx.x; e < (long long)n2 * n2; e += blockDim.x) {
    const int row = (int)(e / n2), col = (int)(e % n2);
    // X[row][col] = B_sigma[col][row]: B row index (a, iz) = col, column index (b, jz) = row
    // transposed: B row index (a, iz) = col, column (b, jz) = row; sym: (a, iz) = row
    const int br = sym ? row : col, bc = sym ? col : row;
    const int a = br / hh, iz = br % hh;
    const int b = bc / hh, jz = bc % hh;
    const double sa = a == 2 ? -1.0 : 1.0, sb = b == 2 ? -1.0 : 1.0;
    const bool vr = (iz < h) || (sig * sa > 0.0);
    const bool vc = (jz < h) || (sig * sb > 0.0);
    double2 val = make_double2(0.0, 0.0);
    if (!vr || !vc) {
      if (row == col) val = make_double2(1.0, 0.0);
    } else {
      const int cab = comp_index(a, b);
      // B[(a,iz),(b,jz)] = ati delta - lambda_ab(iz - jz)
      double2 t = L[cab * S + (iz - jz) + (nz - 1)];
      val = make_double2(-t.x, -t.y);
      if (a == b && iz == jz) val = cadd(val, ati);
      if (jz < h) {
        const int jm = nz - 1 - jz;
        double2 t2 = L[cab * S + (iz - jm) + (nz - 1)];
        double2 v2 = make_double2(-t2.x, -t2.y);
        if (a == b && iz == jm) v2 = cadd(v2, ati);
        val = cadd(val, cscale(v2, sig * sb));
      }
      if (sym && a == 2) val = make_double2(-val.x, -val.y);
    }
    X[e] = to_c(val, TO{});
  }
}

// Gauss-Jordan step for one trailing column j and the panel [k0, k0 + kb): from the
// column's (row-swapped) pivot-row entries, tv[kk] are the multiples of the panel's
// eliminated columns it receives and aK its new pivot-row entries.
// Column j against the panel's NB pivot rows k0 .. k0 + kb - 1 (already swapped into place):
// the multipliers t_kk that the panel's pivot steps apply to column j.  Step kk scales the
// pivot-row entry by 1 / pivot and removes it from the later pivot rows' entries; earlier
// pivot rows' entries are not needed for the multipliers and are left alone.
template <int NB, typename V>
__device__ __forceinline__ void gj_col_mult(const V *A, int n, int j, int k0, int kb, const V *F,
                                            const V *ipv, V (&a)[NB]) {
  using R = typename RealOf<V>::type;
#pragma unroll
  for (int kk = 0; kk < NB; ++kk)
    a[kk] = kk < kb ? A[(long long)(k0 + kk) * n + j] : mk<R>((R)0, (R)0);
#pragma unroll
  for (int kk = 0; kk < NB; ++kk) {
    if (kk >= kb) continue;
    const V t = cmul(a[kk], ipv[kk]);
    a[kk] = t;
#pragma unroll
    for (int k2 = kk + 1; k2 < NB; ++k2)
      if (k2 < kb) a[k2] = csub(a[k2], cmul(F[(k0 + k2) * NB + kk], t));
  }
}

// The pivot rows' final entries in column j from its multipliers (in place): row k0 + kk ends
// as t_kk minus the later steps' multiples of it, t_kk - sum_{kk' > kk} F[k0 + kk][kk'] t_kk'.
template <int NB, typename V>
__device__ __forceinline__ void gj_pivot_vals(int k0, int kb, const V *F, V (&a)[NB]) {
#pragma unroll
  for (int kk = 0; kk < NB; ++kk) {
    if (kk >= kb) continue;
#pragma unroll
    for (int k2 = kk + 1; k2 < NB; ++k2)
      if (k2 < kb) a[kk] = csub(a[kk], cmul(F[(k0 + kk) * NB + k2], a[k2]));
  }
}

constexpr int kGJMaxOrder = 768;  // the largest half-block order, 3 * 256
constexpr size_t kLdsMax = 160 * 1024;  // LDS of one gfx950 CU, the most one workgroup can take
constexpr int kGJThreads = 256;

// Batched in-place inverse of row-major n x n complex matrices (FP64 or FP32), one workgroup each
// (MINW: minimum waves per SIMD the register allocation must allow):
// Gauss-Jordan elimination with partial pivoting, blocked by NB columns.  For each panel of
// NB columns the pivot steps run on rows held in registers (thread t owns rows t + r NT,
// r < RPT); per step a wave-shuffle argmax picks the pivot, the pivot row and the old row k
// pass through LDS, and the multipliers F (n x NB) are kept in LDS.  The other columns then
// receive the panel's row swaps, a short recurrence over the NB pivot rows and a rank-NB
// update of the remaining rows.  Column interchanges are undone at the end.  A zero pivot
// sets flag[0].
template <int NB, int NT, int RPT, typename V, int MINW = 1>
__global__ void __launch_bounds__(NT, MINW) k_gj_inverse(V *mats, int n, int *flag) {
  using R = typename RealOf<V>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *F = reinterpret_cast<V *>(smem_raw);                     // [n][NB]
  int *pivall = reinterpret_cast<int *>(F + (size_t)n * NB);  // [n]
  __shared__ V ipv_s[NB], prow[NB], krow[NB];
  __shared__ R red_v[NT / 64];
  __shared__ int red_i[NT / 64];
  const int tid = threadIdx.x;
  V *A = mats + (long long)blockIdx.x * n * n;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = min(NB, n - k0);
    V rv[RPT][NB];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * NT;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        rv[r][c] = (i < n && c < kb) ? A[(long long)i * n + k0 + c] : mk<R>((R)0, (R)0);
    }
    for (int e = tid; e < n * NB; e += NT) F[e] = mk<R>((R)0, (R)0);
    __syncthreads();
    for (int kk = 0; kk < kb; ++kk) {
      const int k = k0 + kk;
      // pivot: argmax |row i, column kk| over rows i >= k, ties to the smallest row
      R bv = (R)-1;
      int bi = n;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = tid + r * NT;
        V v = rv[r][0];
#pragma unroll
        for (int c = 1; c < NB; ++c)
          if (c == kk) v = rv[r][c];
        const R m2 = v.x * v.x + v.y * v.y;
        if (i < n && i >= k && m2 > bv) { bv = m2; bi = i; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const R ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if ((tid & 63) == 0) {
        red_v[tid >> 6] = bv;
        red_i[tid >> 6] = bi;
      }
      __syncthreads();
      bv = red_v[0];
      int pr = red_i[0];
#pragma unroll
      for (int w = 1; w < NT / 64; ++w)
        if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < pr)) { bv = red_v[w]; pr = red_i[w]; }
      // publish the pivot row and the old row k; the multipliers of earlier panel columns
      // follow the swap
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = tid + r * NT;
        if (i == pr)
#pragma unroll
          for (int c = 0; c < NB; ++c) prow[c] = rv[r][c];
        if (i == k)
#pragma unroll
          for (int c = 0; c < NB; ++c) krow[c] = rv[r][c];
      }
      if (tid < kk && pr != k) {
        const V t = F[k * NB + tid];
        F[k * NB + tid] = F[pr * NB + tid];
        F[pr * NB + tid] = t;
      }
      __syncthreads();
      V pv = prow[0];
#pragma unroll
      for (int c = 1; c < NB; ++c)
        if (c == kk) pv = prow[c];
      const R pm = pv.x * pv.x + pv.y * pv.y;
      const V ipv = pm > (R)0 ? mk<R>(pv.x / pm, -pv.y / pm) : mk<R>((R)0, (R)0);
      if (tid == 0) {
        pivall[k] = pr;
        ipv_s[kk] = ipv;
        if (pm == (R)0) atomicExch(flag, 1);
      }
      // swap rows k and pr, scale the pivot row, eliminate column kk from the other rows
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = tid + r * NT;
        if (i >= n) continue;
        if (i == k) {
#pragma unroll
          for (int c = 0; c < NB; ++c) rv[r][c] = (c == kk) ? ipv : cmul(prow[c], ipv);
          F[k * NB + kk] = mk<R>((R)0, (R)0);
        } else {
          if (i == pr)
#pragma unroll
            for (int c = 0; c < NB; ++c) rv[r][c] = krow[c];
          V f = rv[r][0];
#pragma unroll
          for (int c = 1; c < NB; ++c)
            if (c == kk) f = rv[r][c];
          F[i * NB + kk] = f;
          const V fi = cmul(f, ipv);
#pragma unroll
          for (int c = 0; c < NB; ++c)
            rv[r][c] = (c == kk) ? mk<R>(-fi.x, -fi.y) : csub(rv[r][c], cmul(fi, prow[c]));
        }
      }
      // the next step writes prow / krow only after its first barrier, which every thread
      // reaches after finishing this step
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * NT;
      if (i < n)
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < kb) A[(long long)i * n + k0 + c] = rv[r][c];
    }
    // Trailing columns, in three barrier-separated phases so that no pivot-row value is read
    // after it has been replaced: (A) the panel's row swaps, one thread per column; (B) kRG
    // threads per column each form the column's NB multipliers (a short recurrence over the
    // pivot rows) and update their share of the other rows, sixteen rows of loads in flight;
    // (C) one thread per column forms them again and stores the pivot rows' final entries.
    __syncthreads();
    constexpr int kRG = 4;
    const int ncol = n - kb;
    for (int jj = tid; jj < ncol; jj += NT) {
      const int j = jj < k0 ? jj : jj + kb;
      for (int kk = 0; kk < kb; ++kk) {
        const int k = k0 + kk, pr = pivall[k];
        if (pr != k) {
          V t = A[(long long)k * n + j];
          A[(long long)k * n + j] = A[(long long)pr * n + j];
          A[(long long)pr * n + j] = t;
        }
      }
    }
    __syncthreads();
    const int rows_per = (n + kRG - 1) / kRG;
    for (int w = tid; w < kRG * ncol; w += NT) {
      const int cgrp = w / ncol, jj = w - cgrp * ncol;
      const int j = jj < k0 ? jj : jj + kb;
      V tv[NB];
      gj_col_mult<NB, V>(A, n, j, k0, kb, F, ipv_s, tv);
      const int i0 = cgrp * rows_per, i1 = min(n, i0 + rows_per);
      for (int ib = i0; ib < i1; ib += 16) {
        V av[16];
#pragma unroll
        for (int u = 0; u < 16; ++u)
          av[u] = ib + u < i1 ? A[(long long)(ib + u) * n + j] : mk<R>((R)0, (R)0);
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int i = ib + u;
          if (i >= i1 || (i >= k0 && i < k0 + kb)) continue;
          V acc = av[u];
#pragma unroll
          for (int kk = 0; kk < NB; ++kk) acc = csub(acc, cmul(F[i * NB + kk], tv[kk]));
          A[(long long)i * n + j] = acc;
        }
      }
    }
    __syncthreads();
    for (int jj = tid; jj < ncol; jj += NT) {
      const int j = jj < k0 ? jj : jj + kb;
      V aK[NB];
      gj_col_mult<NB, V>(A, n, j, k0, kb, F, ipv_s, aK);
      gj_pivot_vals<NB, V>(k0, kb, F, aK);
#pragma unroll
      for (int kk = 0; kk < NB; ++kk)
        if (kk < kb) A[(long long)(k0 + kk) * n + j] = aK[kk];
    }
    __syncthreads();
  }
  // undo the column interchanges, last first (each thread owns whole rows)
  for (int i = tid; i < n; i += NT) {
    for (int k = n - 1; k >= 0; --k) {
      const int pr = pivall[k];
      if (pr != k) {
        V t = A[(long long)i * n + k];
        A[(long long)i * n + k] = A[(long long)i * n + pr];
        A[(long long)i * n + pr] = t;
      }
    }
  }
}

// Launch k_gj_inverse with the panel width and rows per thread for order n: 16-column panels
// up to n = 512 (256 threads, or 512 above n = 256, one row each), 8 columns above (three rows
// per thread), in either precision.  Wider panels mean fewer passes over the matrix but more
// LDS per workgroup: 32-column FP32 panels, which fit, ran slower (39.7 vs 21.8 ms at order
// 192, 927 vs 837 ms at order 384 for a 256^3 build) because fewer workgroups share a CU.
template <typename V> static int gj_nb(int n) { return n <= 2 * kGJThreads ? 16 : 8; }
template <typename V> static size_t gj_lds(int n) {
  return sizeof(V) * (size_t)n * gj_nb<V>(n) + sizeof(int) * n;
}
template <typename V> static void gj_launch(dda_problem *p, V *mats, long long cnt, int n) {
  const size_t lds = gj_lds<V>(n);
  if (n <= kGJThreads) {
    auto fn = k_gj_inverse<16, kGJThreads, 1, V>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(kGJThreads), lds, p->st, mats, n, p->dflag);
  } else if (n <= 2 * kGJThreads) {
    // FP32: at least 4 waves per SIMD (128 VGPRs, a 4-register spill) fits two 512-thread
    // workgroups on a CU instead of one: 837 -> 617 ms at order 384 (a 256^3 build).  The same
    // bound costs FP64, and the 256-thread kernels, more than it gains.
    auto fn = k_gj_inverse<16, 2 * kGJThreads, 1, V, sizeof(V) == sizeof(float2) ? 4 : 1>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(2 * kGJThreads), lds, p->st, mats, n, p->dflag);
  } else {
    auto fn = k_gj_inverse<8, kGJThreads, 3, V>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(kGJThreads), lds, p->st, mats, n, p->dflag);
  }
  HIPCHK(hipGetLastError());
}

// 16 x 16 x 4 matrix instruction of each precision.  Lane l = r + 16 q supplies A[r][q] and
// B[q][r]; item m of its result holds D[row(q, m)][r].
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of D held in item m of a lane of k-slot q (column = lane % 16)
  static __device__ __forceinline__ int row(int q, int m) { return q + 4 * m; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int q, int m) { return 4 * q + m; }
};

// Gauss-Jordan with partial pivoting on the NB x 2NB block [A_KK | I] in aug, by the 64 lanes
// of one wave (lane = tid < 64): on return aug[.][NB, 2NB) holds G = A_KK^{-1} for the
// leading kb x kb block.  A pivot whose squared modulus falls below tiny times the block's
// largest sets flag[1].
template <int NB, typename V, typename R>
__device__ __forceinline__ void sweep_gj_wave(V (*aug)[2 * NB], int kb, int tid, int *flag, R tiny) {
  R m = (R)0;
  for (int e = tid; e < kb * kb; e += 64) {
    const V v = aug[e / kb][e % kb];
    m = fmax(m, v.x * v.x + v.y * v.y);
  }
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  __builtin_amdgcn_wave_barrier();
  for (int kk = 0; kk < kb; ++kk) {
    // pivot row: largest |aug[r][kk]| over r >= kk (lanes < 16 hold the candidates)
    R bv = (R)-1;
    int bi = kk;
    if (tid >= kk && tid < kb) {
      const V v = aug[tid][kk];
      bv = v.x * v.x + v.y * v.y;
      bi = tid;
    }
    for (int off = 32; off > 0; off >>= 1) {
      const R ov = __shfl_xor(bv, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ov > bv || (ov == bv && oi < bi)) {
        bv = ov;
        bi = oi;
      }
    }
    if (!(bv > tiny * m) && tid == 0) atomicExch(flag + 1, 1);
    __builtin_amdgcn_wave_barrier();
    // swap rows kk and bi, scale the pivot row
    if (tid < 2 * NB) {
      const V a = aug[kk][tid], b = aug[bi][tid];
      aug[bi][tid] = a;
      aug[kk][tid] = b;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    const V pv = aug[kk][kk];
    const R pm = pv.x * pv.x + pv.y * pv.y;
    const V ipv = pm > (R)0 ? mk<R>(pv.x / pm, -pv.y / pm) : mk<R>((R)0, (R)0);
    __builtin_amdgcn_wave_barrier();
    if (tid < 2 * NB) aug[kk][tid] = cmul(aug[kk][tid], ipv);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    // eliminate column kk from the other rows: lane handles columns c = lane % 32, rows
    // r = lane / 32 + 2 q
    V f[NB / 2], pr;
    const int c = tid & 31, r0 = tid >> 5;
    pr = c < 2 * NB ? aug[kk][c] : mk<R>((R)0, (R)0);
#pragma unroll
    for (int q = 0; q < NB / 2; ++q) f[q] = aug[r0 + 2 * q][kk];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int q = 0; q < NB / 2; ++q) {
      const int r = r0 + 2 * q;
      if (r != kk && c < 2 * NB) aug[r][c] = csub(aug[r][c], cmul(f[q], pr));
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
  }
}

// Batched inverse of complex symmetric n x n matrices (B^T = B, FP64 or FP32) by the blocked
// symmetric sweep, one workgroup each: Gauss-Jordan elimination without row exchanges between
// panels, which keeps every intermediate matrix symmetric, so only the upper triangle (row
// major, column j >= row i) is read and written, half the passes over the matrix that
// k_gj_inverse makes.  For each panel K of NB pivots:
//   G = A_KK^{-1} (Gauss-Jordan with partial pivoting inside the NB x NB block, on [A_KK | I]),
//   U_i = A_iK G for the rows i outside K,
//   A_ij -= U_i A_Kj (i, j outside K), A_iK = U_i, A_KK = -G,
// after which the upper triangle holds -B^{-1}.  A diagonal block whose pivot falls below
// 1e-13 (FP64) or 1e-6 (FP32) of its largest entry sets flag[1]: the caller then inverts the
// same blocks with k_gj_inverse (tiny2 is the squared bound).
template <int NB, int NT, typename V>
__global__ void __launch_bounds__(NT) k_sym_sweep(V *mats, int n, int *flag, double tiny2) {
  using R = typename RealOf<V>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *Pn = reinterpret_cast<V *>(smem_raw);  // [n][NB] panel columns A_iK before the panel
  V *Un = Pn + (size_t)n * NB;              // [n][NB] U_i
  __shared__ V aug[NB][2 * NB];             // [A_KK | I] -> [I | G]
  const int tid = threadIdx.x;
  V *A = mats + (long long)blockIdx.x * n * n;
  const R tiny = (R)tiny2;  // squared relative pivot bound
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kb = min(NB, n - k0), k1 = k0 + kb;
    // the panel's columns: rows above the block and the block by rows, rows below by columns
    for (int e = tid; e < k1 * NB; e += NT) {
      const int i = e / NB, c = e - i * NB, k = k0 + c;
      Pn[e] = c < kb ? (i <= k ? A[(long long)i * n + k] : A[(long long)k * n + i]) : mk<R>((R)0, (R)0);
    }
    for (int e = tid; e < (n - k1) * NB; e += NT) {
      const int c = e / (n - k1), i = k1 + (e - c * (n - k1));
      Pn[i * NB + c] = c < kb ? A[(long long)(k0 + c) * n + i] : mk<R>((R)0, (R)0);
    }
    __syncthreads();
    // G by one wave: Gauss-Jordan with partial pivoting on [A_KK | I]
    if (tid < 64) {
      for (int e = tid; e < NB * 2 * NB; e += 64) {
        const int r = e / (2 * NB), c = e - r * 2 * NB;
        V v = mk<R>((R)0, (R)0);
        if (c < NB) v = (r < kb && c < kb) ? Pn[(k0 + r) * NB + c] : mk<R>(r == c ? (R)1 : (R)0, (R)0);
        else v = mk<R>(c - NB == r ? (R)1 : (R)0, (R)0);
        aug[r][c] = v;
      }
      sweep_gj_wave<NB>(aug, kb, tid, flag, tiny);
    }
    __syncthreads();
    // U = A_iK G for the rows outside the block
    for (int e = tid; e < n * NB; e += NT) {
      const int i = e / NB, c = e - i * NB;
      V u = mk<R>((R)0, (R)0);
      if (c < kb && (i < k0 || i >= k1))
        for (int cc = 0; cc < kb; ++cc) u = cadd(u, cmul(Pn[i * NB + cc], aug[cc][NB + c]));
      Un[e] = u;
    }
    __syncthreads();
    // the upper triangle in items of up to 16 rows of one column (row block b, column j >= 16 b;
    // consecutive items are consecutive columns of a block, so loads coalesce): trailing
    // update, the panel's entries, the block
    const int nrb = (n + 15) / 16;
    const int items = nrb * n - 8 * nrb * (nrb - 1);  // sum over b of n - 16 b
    for (int w = tid; w < items; w += NT) {
      int b = 0, rem = w;
      while (rem >= n - 16 * b) {
        rem -= n - 16 * b;
        ++b;
      }
      const int j = 16 * b + rem;
      const int i0 = 16 * b, i1 = min(j + 1, i0 + 16);
      V *colj = A + j;
      if (j >= k0 && j < k1) {  // a column of the block: rows above it take U, the block -G
        for (int i = i0; i < i1; ++i)
          colj[(long long)i * n] = i >= k0 ? mk<R>(-aug[i - k0][NB + j - k0].x, -aug[i - k0][NB + j - k0].y)
                                           : Un[i * NB + (j - k0)];
        continue;
      }
      V aj[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) aj[c] = Pn[j * NB + c];
      V av[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) av[u] = i0 + u < i1 ? colj[(long long)(i0 + u) * n] : mk<R>((R)0, (R)0);
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u;
        if (i >= i1) continue;
        V acc;
        if (i >= k0 && i < k1) {
          acc = Un[j * NB + (i - k0)];  // entry (i in K, j below K) is the panel's A_jK, now U_j
        } else {
          acc = av[u];
#pragma unroll
          for (int c = 0; c < NB; ++c) acc = csub(acc, cmul(Un[i * NB + c], aj[c]));
        }
        colj[(long long)i * n] = acc;
      }
    }
    __syncthreads();
  }
}

// The symmetric sweep of k_sym_sweep with 16-pivot panels and every tile product on the matrix
// cores.  The matrix is taken as 16 x 16 tiles (I, J), I <= J, padded to 16 nrb with the
// identity; diagonal tiles are kept whole (both triangles).  For panel K:
//   (1) wave 0 inverts A_KK by pivoted Gauss-Jordan (sweep_gj_wave), while the other waves
//       store the previous panel (A_IK = U_I above the diagonal tile, A_KJ = U_J^T right of it);
//   (2) -U_I = -A_IK G for every I != K, into LDS (16 x 16 x 16 complex products);
//   (3) A_IJ -= U_I A_JK^T over the stored tiles outside row and column K, the tile held in
//       the instruction's accumulators: complex products as four real ones,
//       Re += (-Re U) Re P - (-Im U) Im P,  Im += (-Re U) Im P + (-Im U) Re P;
// then A_KK = -G.  The result, flags and fallback are those of k_sym_sweep.
template <typename T, int NW, bool PAD>
__global__ void __launch_bounds__(64 * NW, 4) k_sym_sweep_mfma(cplx<T> *mats, int n, int *flag, double tiny2) {
  using V = cplx<T>;
  using MF = Mfma<T>;
  using v4 = typename MF::v4;
  constexpr int US = 17;  // row stride of Un (complex entries), padded against bank conflicts
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *Un = reinterpret_cast<V *>(smem_raw);  // [16 nrb][US]: -U_i of the current panel
  __shared__ V aug[16][32];                 // [A_KK | I] -> [I | G]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int nrb = (n + 15) / 16, tiles = nrb * (nrb + 1) / 2;
  V *A = mats + (long long)blockIdx.x * n * n;
  const T tiny = (T)tiny2;
  // entry (row, col) of the identity-padded matrix (PAD: n not a multiple of 16); only stored
  // tiles are addressed.  The load is unconditional (from the matrix's first entry when
  // outside) and the padding is blended in arithmetically (a select would be turned back into
  // a branch around the load), so that loads are not serialised behind branches.
  auto at = [&](int row, int col) -> V {
    if constexpr (!PAD) return A[(long long)row * n + col];
    const bool in = row < n && col < n;
    const V v = A[in ? (long long)row * n + col : 0LL];
    const T w = in ? (T)1 : (T)0, id = (!in && row == col) ? (T)1 : (T)0;
    return mk<T>(v.x * w + id, v.y * w);
  };
  auto put = [&](int row, int col, V v) {
    if (!PAD || (row < n && col < n)) A[(long long)row * n + col] = v;
  };
  for (int K = 0; K <= nrb; ++K) {
    const int Kp = K - 1;  // the previous panel, stored now
    if (wv == 0) {
      if (Kp >= 0)
        for (int e = lane; e < 256; e += 64)
          put(16 * Kp + (e >> 4), 16 * Kp + (e & 15), mk<T>(-aug[e >> 4][16 + (e & 15)].x, -aug[e >> 4][16 + (e & 15)].y));
      if (K < nrb) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        for (int e = lane; e < 512; e += 64) {
          const int a = e >> 5, c = e & 31;
          aug[a][c] = c < 16 ? at(16 * K + a, 16 * K + c) : mk<T>(c - 16 == a ? (T)1 : (T)0, (T)0);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
        __builtin_amdgcn_wave_barrier();
        sweep_gj_wave<16>(aug, 16, lane, flag, tiny);
      }
    } else if (Kp >= 0) {
      for (int e = tid - 64; e < nrb * 256; e += 64 * (NW - 1)) {
        const int I = e >> 8, a = (e >> 4) & 15, b = e & 15;
        if (I < Kp) {
          const V u = Un[(16 * I + a) * US + b];
          put(16 * I + a, 16 * Kp + b, mk<T>(-u.x, -u.y));
        } else if (I > Kp) {
          const V u = Un[(16 * I + b) * US + a];
          put(16 * Kp + a, 16 * I + b, mk<T>(-u.x, -u.y));
        }
      }
    }
    if (K == nrb) break;
    __syncthreads();
    // (2) -U_I = -A_IK G
    for (int I = wv; I < nrb; I += NW) {
      if (I == K) continue;
      v4 ur = {0, 0, 0, 0}, ui = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = 4 * kk + q;
        const V a = at(I < K ? 16 * I + r : 16 * K + k, I < K ? 16 * K + k : 16 * I + r);  // A_IK[r][k]
        const V g = aug[k][16 + r];
        ur = MF::mma(a.x, g.x, ur);
        ur = MF::mma(-a.y, g.y, ur);
        ui = MF::mma(a.x, g.y, ui);
        ui = MF::mma(a.y, g.x, ui);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) Un[(16 * I + MF::row(q, m)) * US + r] = mk<T>(-ur[m], -ui[m]);
    }
    __syncthreads();
    // (3) trailing update of the stored tiles outside row and column K (t = J (J + 1) / 2 + I),
    // each tile's entries and panel operand loaded while the previous tile is multiplied
    auto decode = [&](int t, int &I, int &J) {
      J = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
      while (J * (J + 1) / 2 > t) --J;
      while ((J + 1) * (J + 2) / 2 <= t) ++J;
      I = t - J * (J + 1) / 2;
    };
    auto fetch = [&](int I, int J, v4 &cr, v4 &ci, V (&pj)[4]) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const V c = at(16 * I + MF::row(q, m), 16 * J + r);
        cr[m] = c.x;
        ci[m] = c.y;
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int k = 4 * kk + q;
        pj[kk] = at(J < K ? 16 * J + r : 16 * K + k, J < K ? 16 * K + k : 16 * J + r);  // A_JK[r][k]
      }
    };
    v4 cr, ci;
    V pj[4];
    int I = 0, J = 0;
    if (wv < tiles) {
      decode(wv, I, J);
      fetch(I, J, cr, ci, pj);
    }
    for (int t = wv; t < tiles; t += NW) {
      v4 ncr, nci;
      V npj[4];
      int nI = 0, nJ = 0;
      if (t + NW < tiles) {
        decode(t + NW, nI, nJ);
        fetch(nI, nJ, ncr, nci, npj);
      }
      if (I != K && J != K) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const V nu = Un[(16 * I + r) * US + 4 * kk + q];  // -U_I[r][k]
          cr = MF::mma(nu.x, pj[kk].x, cr);
          cr = MF::mma(-nu.y, pj[kk].y, cr);
          ci = MF::mma(nu.x, pj[kk].y, ci);
          ci = MF::mma(nu.y, pj[kk].x, ci);
          if (kk & 1) __builtin_amdgcn_sched_barrier(0);  // two LDS operands ahead at most
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) put(16 * I + MF::row(q, m), 16 * J + r, mk<T>(cr[m], ci[m]));
      }
      cr = ncr;
      ci = nci;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) pj[kk] = npj[kk];
      I = nI;
      J = nJ;
    }
    __syncthreads();
  }
}

// D = C0 + sgn op(A) op(B) for 16 x 16 complex matrices in LDS (row strides lda, ldb, ldc0, ldd;
// op transposes when ta / tb; C0 may be null or equal to D), on the matrix cores by one wave.
// D must not overlap A or B.
template <typename T>
__device__ __forceinline__ void wave_cmm16(const cplx<T> *A, int lda, bool ta, const cplx<T> *B, int ldb,
                                           bool tb, const cplx<T> *C0, int ldc0, T sgn, cplx<T> *D,
                                           int ldd, int lane) {
  using MF = Mfma<T>;
  using v4 = typename MF::v4;
  using V = cplx<T>;
  const int r = lane & 15, q = lane >> 4;
  v4 dr = {0, 0, 0, 0}, di = {0, 0, 0, 0};
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + q;
    const V a = ta ? A[k * lda + r] : A[r * lda + k];  // op(A)[r][k]
    const V b = tb ? B[r * ldb + k] : B[k * ldb + r];  // op(B)[k][r]
    dr = MF::mma(a.x, b.x, dr);
    dr = MF::mma(-a.y, b.y, dr);
    di = MF::mma(a.x, b.y, di);
    di = MF::mma(a.y, b.x, di);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int row = MF::row(q, m);
    const V c = C0 ? C0[row * ldc0 + r] : mk<T>((T)0, (T)0);
    D[row * ldd + r] = mk<T>(c.x + sgn * dr[m], c.y + sgn * di[m]);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// The streamed sweep with 32-pivot panels (tile columns K0 = 2P and K1 = 2P + 1), which halves
// the passes over the matrix.  The order is padded with the identity to an even number of
// tiles.  The 32 x 32 diagonal block [[A00, A01], [A01^T, A11]] is inverted by wave 0 from its
// two 16 x 16 blocks: G00 = A00^{-1} and G11 = S^{-1} with S = A11 - A01^T W, W = G00 A01, by
// pivoted Gauss-Jordan (sweep_gj_wave, so pivoting and its flag are those of two 16-pivot
// panels), then G01 = -W G11 and G00 += -G01 W^T.  Per panel:
//   (2) -U_I = -[A_IK0 | A_IK1] G for the rows outside the panel, into LDS;
//   (3a) the trailing update A_IJ -= U_I [A_JK0 | A_JK1]^T of the next panel's tiles;
//   (3b) wave 0 stores -G of this panel and inverts the next panel's diagonal block, while the
//        other waves update the remaining tiles (lookahead: the inversion is off the path);
//   (4) A_IK = U_I above the panel, A_KJ = U_J^T right of it.
// Result and flags are those of k_sym_sweep.
template <typename T, int NW, bool PAD>
__global__ void __launch_bounds__(64 * NW, 4) k_sym_sweep_mfma2(cplx<T> *mats, int n, int *flag, double tiny2) {
  using V = cplx<T>;
  using MF = Mfma<T>;
  using v4 = typename MF::v4;
  constexpr int US = 33;  // row stride of Un and Gs (complex entries), padded
  constexpr int TS = 17;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nrb = (n + 15) / 16, nrb2 = nrb + (nrb & 1), tiles = nrb2 * (nrb2 + 1) / 2;
  V *Un = reinterpret_cast<V *>(smem_raw);  // [16 nrb2][US]: -U_i of the current panel
  V *Gs = Un + 16 * nrb2 * US;              // [32][US]: G = A_KK^{-1}
  V *Ws = Gs + 32 * US;                     // [16][TS]: W = G00 A01
  V *A01s = Ws + 16 * TS;                   // [16][TS]
  V *A11s = A01s + 16 * TS;                 // [16][TS]
  __shared__ V aug[16][32];                 // [block | I] -> [I | inverse]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  V *A = mats + (long long)blockIdx.x * n * n;
  const T tiny = (T)tiny2;
  // as in k_sym_sweep_mfma (PAD: n not a multiple of 32): unconditional loads, the identity
  // padding blended in
  auto at = [&](int row, int col) __attribute__((always_inline)) -> V {
    if constexpr (!PAD) return A[(long long)row * n + col];
    const bool in = row < n && col < n;
    const V v = A[in ? (long long)row * n + col : 0LL];
    const T w = in ? (T)1 : (T)0, id = (!in && row == col) ? (T)1 : (T)0;
    return mk<T>(v.x * w + id, v.y * w);
  };
  auto put = [&](int row, int col, V v) __attribute__((always_inline)) {
    if (!PAD || (row < n && col < n)) A[(long long)row * n + col] = v;
  };
  auto sync_wave = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
  };
  // wave 0: G of the panel at tile column K0 into Gs
  auto invert_block = [&](int K0) __attribute__((always_inline)) {
    const int K1 = K0 + 1;
    for (int e = lane; e < 512; e += 64) {
      const int a = e >> 5, c = e & 31;
      aug[a][c] = c < 16 ? at(16 * K0 + a, 16 * K0 + c) : mk<T>(c - 16 == a ? (T)1 : (T)0, (T)0);
    }
    for (int e = lane; e < 256; e += 64) {
      const int a = e >> 4, b = e & 15;
      A01s[a * TS + b] = at(16 * K0 + a, 16 * K1 + b);
      A11s[a * TS + b] = at(16 * K1 + a, 16 * K1 + b);
    }
    sync_wave();
    sweep_gj_wave<16>(aug, 16, lane, flag, tiny);  // G00
    for (int e = lane; e < 256; e += 64) Gs[(e >> 4) * US + (e & 15)] = aug[e >> 4][16 + (e & 15)];
    sync_wave();
    wave_cmm16<T>(Gs, US, false, A01s, TS, false, nullptr, 0, (T)1, Ws, TS, lane);         // W = G00 A01
    wave_cmm16<T>(A01s, TS, true, Ws, TS, false, A11s, TS, (T)-1, &aug[0][0], 32, lane);  // S
    for (int e = lane; e < 256; e += 64) aug[e >> 4][16 + (e & 15)] = mk<T>((e >> 4) == (e & 15) ? (T)1 : (T)0, (T)0);
    sync_wave();
    sweep_gj_wave<16>(aug, 16, lane, flag, tiny);  // G11 = S^{-1}
    for (int e = lane; e < 256; e += 64) Gs[(16 + (e >> 4)) * US + 16 + (e & 15)] = aug[e >> 4][16 + (e & 15)];
    sync_wave();
    wave_cmm16<T>(Ws, TS, false, Gs + 16 * US + 16, US, false, nullptr, 0, (T)-1, Gs + 16, US, lane);  // G01
    wave_cmm16<T>(Gs + 16, US, false, Ws, TS, true, Gs, US, (T)-1, Gs, US, lane);  // G00 - G01 W^T
    for (int e = lane; e < 256; e += 64) Gs[(16 + (e >> 4)) * US + (e & 15)] = Gs[(e & 15) * US + 16 + (e >> 4)];
  };
  // A_IJ -= U_I [A_JK0 | A_JK1]^T for one tile (I, J outside the panel at K0); cr / ci hold
  // the tile's entries on entry
  auto update = [&](int I, int J, int K0, v4 &cr, v4 &ci) __attribute__((always_inline)) {
    const int K1 = K0 + 1;
    const bool above = J < K0;
    V pj[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 4 * kk + q, Kc = kk < 4 ? K0 : K1, kc = k & 15;
      pj[kk] = at(above ? 16 * J + r : 16 * Kc + kc, above ? 16 * Kc + kc : 16 * J + r);  // A_JK[r][k]
    }
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const V nu = Un[(16 * I + r) * US + 4 * kk + q];  // -U_I[r][k]
      cr = MF::mma(nu.x, pj[kk].x, cr);
      cr = MF::mma(-nu.y, pj[kk].y, cr);
      ci = MF::mma(nu.x, pj[kk].y, ci);
      ci = MF::mma(nu.y, pj[kk].x, ci);
      if (kk & 1) __builtin_amdgcn_sched_barrier(0);  // two LDS operands ahead at most
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) put(16 * I + MF::row(q, m), 16 * J + r, mk<T>(cr[m], ci[m]));
  };
  auto fetch = [&](int I, int J, v4 &cr, v4 &ci) __attribute__((always_inline)) {
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const V c = at(16 * I + MF::row(q, m), 16 * J + r);
      cr[m] = c.x;
      ci[m] = c.y;
    }
  };
  auto decode = [&](int t, int &I, int &J) __attribute__((always_inline)) {
    J = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    while (J * (J + 1) / 2 > t) --J;
    while ((J + 1) * (J + 2) / 2 <= t) ++J;
    I = t - J * (J + 1) / 2;
  };
  const int np = nrb2 / 2;
  if (wv == 0) invert_block(0);
  __syncthreads();
  for (int P = 0; P < np; ++P) {
    const int K0 = 2 * P, K1 = K0 + 1, N0 = K0 + 2, N1 = K0 + 3;  // this panel, the next one
    const bool next = P + 1 < np;
    // (2) -U_I = -[A_IK0 | A_IK1] G
    for (int I = wv; I < nrb2; I += NW) {
      if (I == K0 || I == K1) continue;
      const bool above = I < K0;
      V pa[8];
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) {
        const int k = 4 * kk + q, Kc = kk < 4 ? K0 : K1, kc = k & 15;
        pa[kk] = at(above ? 16 * I + r : 16 * Kc + kc, above ? 16 * Kc + kc : 16 * I + r);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v4 ur = {0, 0, 0, 0}, ui = {0, 0, 0, 0};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const V g = Gs[(4 * kk + q) * US + 16 * h + r];
          ur = MF::mma(pa[kk].x, g.x, ur);
          ur = MF::mma(-pa[kk].y, g.y, ur);
          ui = MF::mma(pa[kk].x, g.y, ui);
          ui = MF::mma(pa[kk].y, g.x, ui);
          if (kk & 1) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) Un[(16 * I + MF::row(q, m)) * US + 16 * h + r] = mk<T>(-ur[m], -ui[m]);
      }
    }
    __syncthreads();
    // (3a) the next panel's tiles: row / column N0 over X, then N1 over X != N0
    if (next) {
      for (int e = wv; e < 2 * nrb2; e += NW) {
        const int h = e >= nrb2, X = e - h * nrb2, Nh = h ? N1 : N0;
        if (X == K0 || X == K1 || (h && X == N0)) continue;
        const int I = min(X, Nh), J = max(X, Nh);
        v4 cr, ci;
        fetch(I, J, cr, ci);
        update(I, J, K0, cr, ci);
      }
    }
    __syncthreads();
    // (3b) wave 0: -G of this panel, then the next panel's G; the others: the remaining tiles
    if (wv == 0) {
      for (int e = lane; e < 768; e += 64) {
        const int blk = e >> 8, a = (e >> 4) & 15, b = e & 15;
        const int gr = blk == 2 ? 16 + a : a, gc = blk == 0 ? b : 16 + b;
        const V g = Gs[gr * US + gc];
        put(16 * (blk == 2 ? K1 : K0) + a, 16 * (blk == 0 ? K0 : K1) + b, mk<T>(-g.x, -g.y));
      }
      if (next) {
        sync_wave();
        invert_block(N0);
      }
    } else {
      auto skip = [&](int I, int J) __attribute__((always_inline)) {
        return I == K0 || I == K1 || J == K0 || J == K1 || (next && (I == N0 || I == N1 || J == N0 || J == N1));
      };
      v4 cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};  // a skipped tile's registers are never used
      int I = 0, J = 0;
      const int w1 = wv - 1;
      if (w1 < tiles) {
        decode(w1, I, J);
        if (!skip(I, J)) fetch(I, J, cr, ci);
      }
      for (int t = w1; t < tiles; t += NW - 1) {
        v4 ncr = {0, 0, 0, 0}, nci = {0, 0, 0, 0};
        int nI = 0, nJ = 0;
        if (t + NW - 1 < tiles) {
          decode(t + NW - 1, nI, nJ);
          if (!skip(nI, nJ)) fetch(nI, nJ, ncr, nci);
        }
        if (!skip(I, J)) update(I, J, K0, cr, ci);
        cr = ncr;
        ci = nci;
        I = nI;
        J = nJ;
      }
    }
    __syncthreads();
    // (4) this panel's other tiles: A_IK = U_I above it, A_KJ = U_J^T right of it
    for (int e = tid; e < nrb2 * 512; e += 64 * NW) {
      const int I = e >> 9, h = (e >> 8) & 1, a = (e >> 4) & 15, b = e & 15;
      const int Kh = h ? K1 : K0;
      if (I < K0) {
        const V u = Un[(16 * I + a) * US + 16 * h + b];
        put(16 * I + a, 16 * Kh + b, mk<T>(-u.x, -u.y));
      } else if (I > K1) {
        const V u = Un[(16 * I + b) * US + 16 * h + a];
        put(16 * Kh + a, 16 * I + b, mk<T>(-u.x, -u.y));
      }
    }
    __syncthreads();
  }
}

// The same sweep with the whole matrix held on chip, for orders up to 192: every stored tile
// (I <= J) lives in the accumulators of one wave for the whole inversion, so the matrix is
// read once and written once.  Wave 0 only inverts the diagonal blocks (it holds no tiles, so
// the pivoting code and the tiles never share registers); slot s of tile wave w = 1 .. NW - 1
// holds tile t = w - 1 + (NW - 1) s, t = J (J + 1) / 2 + I.  Per panel K the owners of row and
// column K copy them to LDS (A_iK by rows; A_KK into the Gauss-Jordan block), wave 0 inverts
// A_KK, the tile waves put -U_I = -A_IK G in LDS and then update their tiles from the two LDS
// panels (A_IJ -= U_I A_JK^T) or replace them (A_IK = U_I, A_KJ = U_J^T, A_KK = -G).  Both
// kinds of wave pass the same four barriers per panel.
template <typename T, int NW, int S>
__global__ void __launch_bounds__(64 * NW) k_sym_sweep_res(cplx<T> *mats, int n, int *flag, double tiny2) {
  using V = cplx<T>;
  using MF = Mfma<T>;
  using v4 = typename MF::v4;
  constexpr int US = 17, NTW = NW - 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int nrb = (n + 15) / 16, tiles = nrb * (nrb + 1) / 2;
  V *Pn = reinterpret_cast<V *>(smem_raw);  // [16 nrb][US]: A_iK of the current panel
  V *Un = Pn + 16 * nrb * US;               // [16 nrb][US]: -U_i
  __shared__ V aug[16][32];                 // [A_KK | I] -> [I | G]
  // the wave index as a scalar, so that the slots' tile coordinates stay in scalar registers
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  if (wv == 0) {
    const T tiny = (T)tiny2;
    for (int K = 0; K < nrb; ++K) {
      __syncthreads();  // (1) A_KK in aug
      sweep_gj_wave<16>(aug, 16, lane, flag, tiny);
      __syncthreads();  // (2) G
      __syncthreads();  // (3) -U
      __syncthreads();  // (4) tiles updated, aug free
    }
    return;
  }
  const int tw = wv - 1;
  V *A = mats + (long long)blockIdx.x * n * n;
  int TI[S], TJ[S];  // the slots' tiles (TI < 0: none)
  v4 cr[S], ci[S];
  {
    const int r = lane & 15, q = lane >> 4;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int t = tw + NTW * s;
      int I = -1, J = 0;
      if (t < tiles) {
        J = (int)((sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
        while (J * (J + 1) / 2 > t) --J;
        while ((J + 1) * (J + 2) / 2 <= t) ++J;
        I = t - J * (J + 1) / 2;
      }
      TI[s] = I;
      TJ[s] = J;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const int row = 16 * I + MF::row(q, m), col = 16 * J + r;
        const bool in = I >= 0 && row < n && col < n;
        const V v = A[in ? (long long)row * n + col : 0LL];  // unconditional, as in k_sym_sweep_mfma
        const T w = in ? (T)1 : (T)0, id = (!in && row == col) ? (T)1 : (T)0;
        cr[s][m] = v.x * w + id;
        ci[s][m] = v.y * w;
      }
      __builtin_amdgcn_sched_barrier(0);  // one slot's loads in flight at a time
    }
  }
  for (int K = 0; K < nrb; ++K) {
    // lane coordinates re-derived each panel, so that no slot keeps LDS addresses of its own
    int r = lane & 15, q = lane >> 4;
    asm volatile("" : "+v"(r), "+v"(q));
    // (1) row and column K to LDS
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int I = TI[s], J = TJ[s];
      if (I < 0) continue;
      if (J == K && I < K) {
#pragma unroll
        for (int m = 0; m < 4; ++m) Pn[(16 * I + MF::row(q, m)) * US + r] = mk<T>(cr[s][m], ci[s][m]);
      } else if (I == K && J > K) {
#pragma unroll
        for (int m = 0; m < 4; ++m) Pn[(16 * J + r) * US + MF::row(q, m)] = mk<T>(cr[s][m], ci[s][m]);
      } else if (I == K && J == K) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          aug[MF::row(q, m)][r] = mk<T>(cr[s][m], ci[s][m]);
          aug[MF::row(q, m)][16 + r] = mk<T>(MF::row(q, m) == r ? (T)1 : (T)0, (T)0);
        }
      }
    }
    __syncthreads();
    __syncthreads();  // (2) wave 0 has inverted A_KK
    // (3) -U_I = -A_IK G
    for (int I = tw; I < nrb; I += NTW) {
      if (I == K) continue;
      v4 ur = {0, 0, 0, 0}, ui = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const V a = Pn[(16 * I + r) * US + 4 * kk + q];
        const V g = aug[4 * kk + q][16 + r];
        ur = MF::mma(a.x, g.x, ur);
        ur = MF::mma(-a.y, g.y, ur);
        ui = MF::mma(a.x, g.y, ui);
        ui = MF::mma(a.y, g.x, ui);
        __builtin_amdgcn_sched_barrier(0);  // registers: every slot's tile is live here
      }
#pragma unroll
      for (int m = 0; m < 4; ++m) Un[(16 * I + MF::row(q, m)) * US + r] = mk<T>(-ur[m], -ui[m]);
    }
    __syncthreads();
    // (4) update or replace the slots' tiles
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int I = TI[s], J = TJ[s];
      if (I < 0) continue;
      if (I != K && J != K) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const V nu = Un[(16 * I + r) * US + 4 * kk + q];  // -U_I[r][k]
          const V pj = Pn[(16 * J + r) * US + 4 * kk + q];  // A_JK[r][k]
          cr[s] = MF::mma(nu.x, pj.x, cr[s]);
          cr[s] = MF::mma(-nu.y, pj.y, cr[s]);
          ci[s] = MF::mma(nu.x, pj.y, ci[s]);
          ci[s] = MF::mma(nu.y, pj.x, ci[s]);
          if (kk & 1) __builtin_amdgcn_sched_barrier(0);
        }
      } else if (I != K) {  // A_IK = U_I
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const V v = Un[(16 * I + MF::row(q, m)) * US + r];
          cr[s][m] = -v.x;
          ci[s][m] = -v.y;
        }
      } else if (J != K) {  // A_KJ = U_J^T
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const V v = Un[(16 * J + r) * US + MF::row(q, m)];
          cr[s][m] = -v.x;
          ci[s][m] = -v.y;
        }
      } else {  // A_KK = -G
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const V v = aug[MF::row(q, m)][16 + r];
          cr[s][m] = -v.x;
          ci[s][m] = -v.y;
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // one slot's operands in registers at a time
    }
    __syncthreads();
  }
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int I = TI[s], J = TJ[s];
    if (I < 0) continue;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int row = 16 * I + MF::row(q, m), col = 16 * J + r;
      if (row < n && col < n) A[(long long)row * n + col] = mk<T>(cr[s][m], ci[s][m]);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Launch the symmetric sweep.  Small orders keep the matrix on chip (k_sym_sweep_res: two
// 16 nrb x 17 panels in LDS; up to 3 stored tiles per tile wave in FP64, order 144, and 6 in
// FP32, order 192; 8 waves per workgroup up to 35 stored tiles, 16 above).  Larger orders
// stream the tiles through HBM once per panel: in FP32 with 32-pivot panels
// (k_sym_sweep_mfma2) where -U of the panel (16 nrb x 33) fits the LDS beside the 32 x 32
// block's work arrays (up to order 512), otherwise with 16-pivot panels (k_sym_sweep_mfma,
// 16 nrb x 17), with 8 waves per workgroup where two workgroups share a CU and 16 where one
// fits.  In FP64 the 32-pivot kernel was measured no faster at order 192 (5.2 vs 5.1 ms per
// launch of 2817 matrices; its operand loads, not its traffic, set its time), so FP64 takes
// 16-pivot panels.  Orders whose 16-pivot panel exceeds the LDS (FP64 above 544) take the
// vector kernel, with 16-pivot panels while its two n x NB panel arrays fit the LDS and 8
// above.  DDA_SWEEP_KERNEL=stream2, =stream or =vector selects a kernel at every order it can
// take.
enum SweepKernel { SW_RES, SW_STREAM2, SW_STREAM, SW_VECTOR };
template <typename V> static size_t sweep_panel_lds(int n) { return (size_t)16 * ((n + 15) / 16) * 17 * sizeof(V); }
template <typename V> static size_t sweep_panel2_lds(int n) {
  const int nrb = (n + 15) / 16, nrb2 = nrb + (nrb & 1);
  return ((size_t)16 * nrb2 * 33 + 32 * 33 + 3 * 16 * 17) * sizeof(V);
}
template <typename V> static SweepKernel sweep_kernel(int n) {
  const char *e = getenv("DDA_SWEEP_KERNEL");
  const size_t aug = 16 * 32 * sizeof(V);
  const bool stream_ok = sweep_panel_lds<V>(n) + aug <= kLdsMax;
  const bool stream2_ok = sweep_panel2_lds<V>(n) + aug <= kLdsMax;
  if (e && strcmp(e, "vector") == 0) return SW_VECTOR;
  if (e && strcmp(e, "stream") == 0 && stream_ok) return SW_STREAM;
  if (e && strcmp(e, "stream2") == 0 && stream2_ok) return SW_STREAM2;
  const int nrb = (n + 15) / 16;
  const bool fp64 = sizeof(V) == sizeof(double2);
  if (nrb * (nrb + 1) / 2 <= 15 * (fp64 ? 3 : 6)) return SW_RES;
  return (stream2_ok && !fp64) ? SW_STREAM2 : stream_ok ? SW_STREAM : SW_VECTOR;
}
template <typename V> static int sweep_nb(int n) {
  return (size_t)2 * n * 16 * sizeof(V) <= 96 * 1024 ? 16 : 8;
}
template <typename V> static size_t sweep_lds(int n) {
  switch (sweep_kernel<V>(n)) {
    case SW_RES: return 2 * sweep_panel_lds<V>(n);
    case SW_STREAM2: return sweep_panel2_lds<V>(n);
    case SW_STREAM: return sweep_panel_lds<V>(n);
    default: return (size_t)2 * n * sweep_nb<V>(n) * sizeof(V);
  }
}
template <typename T, int NW>
static void sweep_res_launch(dda_problem *p, cplx<T> *mats, long long cnt, int n, size_t lds, double tiny2) {
  const int nrb = (n + 15) / 16, slots = (nrb * (nrb + 1) / 2 + NW - 2) / (NW - 1);
  REQUIRE(slots <= 6, DDA_EUNSUPPORTED, "order %d: %d stored tiles per wave", n, slots);
  using Fn = void (*)(cplx<T> *, int, int *, double);
  Fn fn = slots <= 1 ? k_sym_sweep_res<T, NW, 1>
        : slots == 2 ? k_sym_sweep_res<T, NW, 2>
        : slots == 3 ? k_sym_sweep_res<T, NW, 3>
        : slots == 4 ? k_sym_sweep_res<T, NW, 4>
        : slots == 5 ? k_sym_sweep_res<T, NW, 5>
                     : k_sym_sweep_res<T, NW, 6>;
  set_lds_limit((const void *)fn, lds);
  hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(64 * NW), lds, p->st, mats, n, p->dflag, tiny2);
}
template <typename V> static void sweep_launch(dda_problem *p, V *mats, long long cnt, int n) {
  using T = typename RealOf<V>::type;
  const size_t lds = sweep_lds<V>(n);
  // squared relative pivot bound; DDA_SWEEP_FALLBACK=1 flags every block (tests of the fallback)
  double tiny2 = sizeof(V) == sizeof(double2) ? 1e-26 : 1e-12;
  if (const char *e = getenv("DDA_SWEEP_FALLBACK"))
    if (atoi(e) != 0) tiny2 = 1e30;
  const SweepKernel kind = sweep_kernel<V>(n);
  if (kind == SW_RES) {
    const int nrb = (n + 15) / 16;
    if (nrb * (nrb + 1) / 2 <= 7 * 5) sweep_res_launch<T, 8>(p, mats, cnt, n, lds, tiny2);
    else sweep_res_launch<T, 16>(p, mats, cnt, n, lds, tiny2);
  } else if (kind == SW_STREAM2) {
    const bool two = 2 * (lds + 16 * 32 * sizeof(V)) <= kLdsMax, pad = n % 32 != 0;
    auto fn = two ? (pad ? k_sym_sweep_mfma2<T, 8, true> : k_sym_sweep_mfma2<T, 8, false>)
                  : (pad ? k_sym_sweep_mfma2<T, 16, true> : k_sym_sweep_mfma2<T, 16, false>);
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(two ? 512 : 1024), lds, p->st, mats, n, p->dflag, tiny2);
  } else if (kind == SW_STREAM) {
    const bool two = 2 * (lds + 16 * 32 * sizeof(V)) <= kLdsMax, pad = n % 16 != 0;
    auto fn = two ? (pad ? k_sym_sweep_mfma<T, 8, true> : k_sym_sweep_mfma<T, 8, false>)
                  : (pad ? k_sym_sweep_mfma<T, 16, true> : k_sym_sweep_mfma<T, 16, false>);
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(two ? 512 : 1024), lds, p->st, mats, n, p->dflag, tiny2);
  } else {
    auto fn = sweep_nb<V>(n) == 16 ? k_sym_sweep<16, 512, V> : k_sym_sweep<8, 512, V>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)cnt), dim3(512), lds, p->st, mats, n, p->dflag, tiny2);
  }
  HIPCHK(hipGetLastError());
}

__global__ void k_to_f32(const double2 *in, float2 *out, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

static inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

// Element (r, c) of a 16 x 16 tile sits at r + 16 (c % 4) + 64 (c / 4): lane l = r + 16 q of
// a wave reads the tile with four 1 KB loads l + 64 k and receives row r, column 4 k + q, which
// is the A operand of the k-th 16 x 16 x 4 matrix instruction over the tile's columns.
__host__ __device__ __forceinline__ int tile_pos(int r, int c) { return r + 16 * (c & 3) + 64 * (c >> 2); }

// Pack the lower-triangle tiles (I >= J, tile t = I (I + 1) / 2 + J) of `cnt` symmetric
// row-major n2 x n2 matrices into out + m0 * tiles * 256; entries beyond n2 are zero.
// With NEG_UPPER the matrices hold -B^{-1} in their upper triangle only (k_sym_sweep).
template <typename TI, typename TO, bool NEG_UPPER>
__global__ void k_pack_sym(const TI *Y, TO *out, long long m0, int n2, int ntr) {
  const long long tiles = (long long)ntr * (ntr + 1) / 2;
  const TI *Ym = Y + (long long)blockIdx.x * n2 * n2;
  TO *o = out + (m0 + blockIdx.x) * tiles * 256;
  for (long long e = threadIdx.x; e < tiles * 256; e += blockDim.x) {
    const long long t = e >> 8;
    const int w = (int)(e & 255);
    int I = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while ((long long)I * (I + 1) / 2 > t) --I;
    while ((long long)(I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = (int)(t - (long long)I * (I + 1) / 2);
    // invert tile_pos: w = r + 16 (c % 4) + 64 (c / 4)
    const int r = w & 15, c = 4 * (w >> 6) + ((w >> 4) & 3);
    const int row = 16 * I + r, col = 16 * J + c;
    double2 v = make_double2(0.0, 0.0);
    if (row < n2 && col < n2) {
      if (NEG_UPPER) {
        v = to_d(Ym[(long long)min(row, col) * n2 + max(row, col)]);
        v = make_double2(-v.x, -v.y);
      } else {
        v = to_d(Ym[(long long)row * n2 + col]);
      }
    }
    o[t * 256 + w] = to_c(v, TO{});
  }
}



void precond_free(dda_problem *p) {
  if (p->binv64) (void)hipFree(p->binv64);
  if (p->binv32) (void)hipFree(p->binv32);
  if (p->pdelta) (void)hipFree(p->pdelta);
  if (p->pdt) (void)hipFree(p->pdt);
  if (p->pdz) (void)hipFree(p->pdz);
  p->binv64 = nullptr;
  p->binv32 = nullptr;
  p->pdelta = p->pdt = p->pdz = nullptr;
  p->prec_built = 0;
}

// Delta[c] = 1/alpha_j - alpha~^{-1} at the voxel j of compact entry c: what the circulant
// preconditioner's constant diagonal misses of the true diagonal D (Sec. 1, P = D~ + C)
__global__ void k_diag_delta(const double2 *eps, const int *vox, long long nocc, double kd,
                             double s_bar, double2 ati, double2 *delta) {
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c < nocc) delta[c] = csub(ldr_alpha_inv(eps[vox[c]], kd, s_bar), ati);
}

// t = s_r x - Delta z on compact [nrhs][3][nocc] vectors, s_r = xscale[r * kMaxM] (or 1);
// blockIdx.y = 3 r + component
__global__ void k_diag_resid(const double2 *x, const double2 *z, const double2 *delta,
                             double2 *t, long long nocc, const double *xscale, const int *act) {
  if (act && !act[blockIdx.y / 3]) return;
  const long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (c >= nocc) return;
  const long long i = blockIdx.y * nocc + c;
  double2 xv = x[i];
  if (xscale) xv = cscale(xv, xscale[(blockIdx.y / 3) * kMaxM]);
  t[i] = csub(xv, cmul(delta[c], z[i]));
}

// The circulant-plus-diagonal data (opt.diag_steps > 0), after the circulant part is built.
static void diag_setup(dda_problem *p, double s_bar) {
  if (p->opt.diag_steps <= 0) return;
  try {
    const size_t vec = sizeof(double2) * (size_t)p->R * 3 * (size_t)p->nocc;
    HIPCHK(hipMalloc(&p->pdelta, sizeof(double2) * (size_t)std::max<long long>(p->nocc, 1)));
    HIPCHK(hipMalloc(&p->pdt, std::max<size_t>(vec, 16)));
    HIPCHK(hipMalloc(&p->pdz, std::max<size_t>(vec, 16)));
    if (p->nocc > 0) {
      hipLaunchKernelGGL(k_diag_delta, dim3(nblk(p->nocc, 256)), dim3(256), 0, p->st, p->eps,
                         p->vox, p->nocc, p->k * p->d, s_bar, p->ati, p->pdelta);
      HIPCHK(hipGetLastError());
    }
  } catch (...) {
    precond_free(p);
    throw;
  }
}

static void precond1_build(dda_problem *p);

// The preconditioner's constant diagonal alpha~^{-1} (Sec. 1, Sec. 3.1) from the occupied
// voxels, by opt.alpha_avg: 1/alpha of the mean permittivity; the mean of 1/alpha (exact from
// the setup's means of eps and of (eps + 2)/(eps - 1)); or 1/alpha of the most frequent
// permittivity, ties to the smallest value (real part first).
static double2 alpha_tilde_inv(dda_problem *p, double s_bar) {
  const double kd = p->k * p->d;
  if (p->opt.alpha_avg == 1) return ldr_alpha_inv_q(p->cm_mean, p->eps_mean, kd, s_bar);
  if (p->opt.alpha_avg != 2) return ldr_alpha_inv(p->eps_mean, kd, s_bar);
  std::vector<uint8_t> m(p->N);
  std::vector<double2> e(p->N);
  HIPCHK(hipMemcpyAsync(m.data(), p->mask, p->N, hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipMemcpyAsync(e.data(), p->eps, sizeof(double2) * p->N, hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  std::map<std::pair<double, double>, long long> count;
  for (long long v = 0; v < p->N; ++v)
    if (m[v]) ++count[std::make_pair(e[v].x, e[v].y)];
  std::pair<double, double> best{0.0, 0.0};
  long long top = -1;
  for (const auto &kv : count)  // ascending values: a tie keeps the smallest
    if (kv.second > top) {
      top = kv.second;
      best = kv.first;
    }
  return ldr_alpha_inv(make_double2(best.first, best.second), kd, s_bar);
}

template <typename T>
static void pc_apply(dda_problem *p, int nrhs, const double2 *x, double2 *y, const cplx<T> *binv,
                     const double *xscale);

void precond_build(dda_problem *p, double s_bar) {
  precond_free(p);
  if (p->opt.precond == 1) {
    p->ati = alpha_tilde_inv(p, s_bar);
    precond1_build(p);
    diag_setup(p, s_bar);
    return;
  }
  const int nx = p->nx, ny = p->ny, nz = p->pbz;  // the dense level's extent
  p->ati = alpha_tilde_inv(p, s_bar);
  p->hh = (nz + 1) / 2;
  p->n2 = 3 * p->hh;
  p->umx = nx / 2 + 1;
  p->umy = ny / 2 + 1;
  const long long U = (long long)p->umx * p->umy;
  const long long nmat = 2 * U;
  const long long msz = (long long)p->n2 * p->n2;
  const int fp32 = p->opt.precision == 1;
  p->psym = nz % 2 == 0 ? 1 : 0;
  p->ntr = (p->n2 + 15) / 16;
  const long long per = p->psym ? (long long)p->ntr * (p->ntr + 1) / 2 * 256 : msz;  // stored
  const size_t final_bytes = (size_t)nmat * per * (fp32 ? sizeof(float2) : sizeof(double2));
  size_t freeb = 0, totb = 0;
  HIPCHK(hipMemGetInfo(&freeb, &totb));
  REQUIRE(final_bytes < (size_t)(0.85 * (double)freeb), DDA_ENOMEM,
          "preconditioner blocks need %.2f GB, %.2f GB free", final_bytes / 1e9, freeb / 1e9);

  // generator and its 2-D DFT
  const long long S = 2LL * nz - 1;
  const long long gtot = 6 * S * (long long)nx * ny;
  double2 *gen = nullptr, *scratch = nullptr;
  HIPCHK(hipMalloc(&gen, sizeof(double2) * gtot));
  try {
    hipLaunchKernelGGL(k_chan_gen, dim3(nblk(S * nx * ny, 256)), dim3(256), 0, p->st, gen, nx, ny,
                       nz, p->k, p->d);
    HIPCHK(hipGetLastError());
    fft_rows_plain(p, p->ux, gen, 6 * S * ny, 0);
    fft_strided_plain(p, p->uy, gen, 6 * S, nx, 0);

    if (fp32) HIPCHK(hipMalloc(&p->binv32, final_bytes));
    else HIPCHK(hipMalloc(&p->binv64, final_bytes));
    // Blocks are assembled and inverted in the precision they are applied in (FP32 blocks by
    // FP32 Gauss-Jordan); symmetric halves go through scratch to be packed into tiles, full
    // (odd nz) ones are inverted in place.
    const size_t esz = fp32 ? sizeof(float2) : sizeof(double2);
    long long chunk = nmat;
    if (p->psym) {
      // up to 8 GiB of halves per launch, split evenly: fewer, equal launches leave less of
      // the GPU idle in their last rounds of workgroups (at 128^3 all 8450 halves in one)
      const long long per = std::max<long long>(1, (long long)((8ULL << 30) / (msz * esz)));
      const long long nch = (nmat + per - 1) / per;
      chunk = (nmat + nch - 1) / nch;
      while (hipMalloc(&scratch, esz * chunk * msz) != hipSuccess) {
        (void)hipGetLastError();
        scratch = nullptr;
        REQUIRE(chunk > 1, DDA_ENOMEM, "no device memory for one preconditioner block");
        chunk = (chunk + 1) / 2;
      }
    }
    const size_t lds_asm = sizeof(double2) * 6 * S;
    set_lds_limit((const void *)k_assemble<double2>, lds_asm);
    set_lds_limit((const void *)k_assemble<float2>, lds_asm);
    const size_t lds_gj = std::max(fp32 ? gj_lds<float2>(p->n2) : gj_lds<double2>(p->n2),
                                   p->psym ? (fp32 ? sweep_lds<float2>(p->n2) : sweep_lds<double2>(p->n2)) : 0);
    REQUIRE(p->n2 <= kGJMaxOrder, DDA_EUNSUPPORTED, "half-block order %d above %d", p->n2, kGJMaxOrder);
    const size_t lds_cap = std::max(p->lds_max, kLdsMax);
    REQUIRE(lds_gj <= lds_cap && lds_asm <= lds_cap, DDA_EUNSUPPORTED,
            "preconditioner blocks too large for LDS (nz = %d)", nz);
    HIPCHK(hipMemsetAsync(p->dflag, 0, sizeof(int) * 4, p->st));
    // symmetric blocks (even nz) are inverted by the symmetric sweep, unless one of its
    // diagonal blocks needs a row exchange from outside it: then the whole build is redone
    // with pivoted Gauss-Jordan
    bool sweep = p->psym != 0;
    if (const char *e = getenv("DDA_GJ_ONLY")) sweep = sweep && atoi(e) == 0;
    auto run = [&](auto *dst, auto *final_out, long long m0, long long cnt) {
      using V = std::remove_pointer_t<decltype(dst)>;
      {
        KTimer t(&p->prof, p->st, "pc_assemble", (double)esz * cnt * msz);
        hipLaunchKernelGGL(k_assemble<V>, dim3((unsigned)cnt), dim3(256), lds_asm, p->st, gen, dst,
                           m0, nx, ny, nz, p->umx, p->hh, p->n2, p->ati, p->psym);
        HIPCHK(hipGetLastError());
      }
      if (sweep) {
        KTimer t(&p->prof, p->st, "pc_sweep_inverse", esz * cnt * (double)msz);
        sweep_launch<V>(p, dst, cnt, p->n2);
      } else {
        KTimer t(&p->prof, p->st, "pc_gj_inverse", 2.0 * esz * cnt * msz);
        gj_launch<V>(p, dst, cnt, p->n2);
      }
      if (p->psym) {
        using TO = std::remove_pointer_t<decltype(final_out)>;
        auto pk = sweep ? k_pack_sym<V, TO, true> : k_pack_sym<V, TO, false>;
        hipLaunchKernelGGL(pk, dim3((unsigned)cnt), dim3(256), 0, p->st, dst, final_out, m0, p->n2,
                           p->ntr);
        HIPCHK(hipGetLastError());
      }
    };
    int hflag[4] = {0, 0, 0, 0};
    for (int attempt = 0; attempt < 2; ++attempt) {
      for (long long m0 = 0; m0 < nmat; m0 += chunk) {
        const long long cnt = std::min(chunk, nmat - m0);
        if (fp32)
          run(p->psym ? reinterpret_cast<float2 *>(scratch) : p->binv32 + m0 * msz, p->binv32, m0, cnt);
        else
          run(p->psym ? scratch : p->binv64 + m0 * msz, p->binv64, m0, cnt);
      }
      HIPCHK(hipMemcpyAsync(hflag, p->dflag, sizeof(int) * 4, hipMemcpyDeviceToHost, p->st));
      HIPCHK(hipStreamSynchronize(p->st));
      if (!(sweep && hflag[1])) break;
      sweep = false;  // a diagonal block of the sweep needed an outside pivot: Gauss-Jordan
      HIPCHK(hipMemsetAsync(p->dflag, 0, sizeof(int) * 4, p->st));
    }
    p->prec_sweep = sweep ? 1 : 0;
    REQUIRE(hflag[0] == 0, DDA_EDEVICE, "a preconditioner block is singular");
  } catch (...) {
    if (gen) (void)hipFree(gen);
    if (scratch) (void)hipFree(scratch);
    precond_free(p);
    throw;
  }
  HIPCHK(hipFree(gen));
  if (scratch) HIPCHK(hipFree(scratch));
  p->prec_built = 1;
  p->prec_fp32 = fp32;
  diag_setup(p, s_bar);
  // x / y pass shapes of the apply, on the zero Krylov basis
  const int nt = std::min(p->R, 8);
  if (fp32)
    fft_tile_autotune(p, FP_PC_X_FWD, 1, nt,
                      [&] { pc_apply<float>(p, nt, p->V, p->work, p->binv32, nullptr); });
  else
    fft_tile_autotune(p, FP_PC_X_FWD, 0, nt,
                      [&] { pc_apply<double>(p, nt, p->V, p->work, p->binv64, nullptr); });
}

// ----------------------------------------------------------------------------- 1-level

// The 1-level preconditioner C_B of Sec. 3: eq. Chan along x only, so each x mode keeps a
// dense (3 nz ny)^2 block, block-Toeplitz-Toeplitz-block in z and y.
// gen1[c][sz + nz - 1][sy + ny - 1][pbar] = sum over p in {pbar, pbar - nx} of wx(p) K_c(p, sy, sz).
__global__ void k_chan_gen1(double2 *gen, int nx, int ny, int nz, double k, double d) {
  const long long SY = 2LL * ny - 1, SZ = 2LL * nz - 1;
  const long long tot = SZ * SY * nx;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int pb = (int)(idx % nx);
  const int sy = (int)((idx / nx) % SY) - (ny - 1);
  const int sz = (int)(idx / ((long long)nx * SY)) - (nz - 1);
  double2 acc[6];
  for (int c = 0; c < 6; ++c) acc[c] = make_double2(0.0, 0.0);
  const double d3 = d * d * d;
  const int ps[2] = {pb, pb - nx};
  const double wxs[2] = {(double)(nx - pb) / nx, (double)pb / nx};
  for (int u = 0; u < 2; ++u)
    if (wxs[u] != 0.0) green6_chan(ps[u] * d, sy * d, sz * d, k, d3, wxs[u], acc);
  for (int c = 0; c < 6; ++c) gen[c * tot + idx] = acc[c];
}

// X = D(u)^T, row-major, for the unique x modes u in [m0, m0 + count):
// D[(a, iz, iy), (b, jz, jy)] = ati delta - lambda_ab(u; iz - jz, iy - jy), unknown index
// a nz ny + iz ny + iy.
__global__ void k_assemble1(const double2 *lam, double2 *out, long long m0, int nx, int ny, int nz,
                            double2 ati) {
  const long long u = m0 + blockIdx.x;
  const int m = nz * ny, n1 = 3 * m;
  const long long SY = 2LL * ny - 1, SZ = 2LL * nz - 1, tot = SZ * SY * nx;
  double2 *X = out + (long long)blockIdx.x * n1 * n1;
  for (long long e = threadIdx.x; e < (long long)n1 * n1; e += blockDim.x) {
    const int br = (int)(e % n1), bc = (int)(e / n1);  // X[bc][br] = D[br][bc]
    const int a = br / m, rz = (br % m) / ny, ry = br % ny;
    const int b = bc / m, cz = (bc % m) / ny, cy = bc % ny;
    const double2 t = lam[comp_index(a, b) * tot + ((long long)(rz - cz + nz - 1) * SY + (ry - cy + ny - 1)) * nx + u];
    double2 val = make_double2(-t.x, -t.y);
    if (br == bc) val = cadd(val, ati);
    X[e] = val;
  }
}

static void precond1_build(dda_problem *p) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const int n1 = 3 * nz * ny;
  REQUIRE(n1 <= kGJMaxOrder, DDA_EUNSUPPORTED,
          "1-level blocks of order 3 nz ny = %d above %d (use the 2-level preconditioner)", n1,
          kGJMaxOrder);
  p->n2 = n1;
  p->umx = nx / 2 + 1;
  p->umy = 1;
  p->psym = 0;
  const long long nmat = p->umx, msz = (long long)n1 * n1;
  const int fp32 = p->opt.precision == 1;
  const size_t final_bytes = (size_t)nmat * msz * (fp32 ? sizeof(float2) : sizeof(double2));
  size_t freeb = 0, totb = 0;
  HIPCHK(hipMemGetInfo(&freeb, &totb));
  REQUIRE(final_bytes < (size_t)(0.85 * (double)freeb), DDA_ENOMEM,
          "preconditioner blocks need %.2f GB, %.2f GB free", final_bytes / 1e9, freeb / 1e9);
  const long long rows = 6LL * (2 * nz - 1) * (2 * ny - 1);
  double2 *gen = nullptr, *scratch = nullptr;
  HIPCHK(hipMalloc(&gen, sizeof(double2) * rows * nx));
  try {
    hipLaunchKernelGGL(k_chan_gen1, dim3(nblk(rows / 6 * nx, 256)), dim3(256), 0, p->st, gen, nx, ny,
                       nz, p->k, p->d);
    HIPCHK(hipGetLastError());
    fft_rows_plain(p, p->ux, gen, rows, 0);
    if (fp32) HIPCHK(hipMalloc(&p->binv32, final_bytes));
    else HIPCHK(hipMalloc(&p->binv64, final_bytes));
    long long chunk = nmat;
    if (fp32) {
      chunk = std::max<long long>(1, (long long)((1ULL << 31) / (msz * sizeof(double2))));
      chunk = std::min(chunk, nmat);
      HIPCHK(hipMalloc(&scratch, sizeof(double2) * chunk * msz));
    }
    REQUIRE(gj_lds<double2>(n1) <= std::max(p->lds_max, kLdsMax), DDA_EUNSUPPORTED,
            "1-level blocks too large for LDS (order %d)", n1);
    HIPCHK(hipMemsetAsync(p->dflag, 0, sizeof(int) * 4, p->st));
    for (long long m0 = 0; m0 < nmat; m0 += chunk) {
      const long long cnt = std::min(chunk, nmat - m0);
      double2 *dst = fp32 ? scratch : p->binv64 + m0 * msz;
      {
        KTimer t(&p->prof, p->st, "pc_assemble", 16.0 * cnt * msz);
        hipLaunchKernelGGL(k_assemble1, dim3((unsigned)cnt), dim3(256), 0, p->st, gen, dst, m0, nx, ny,
                           nz, p->ati);
        HIPCHK(hipGetLastError());
      }
      {
        KTimer t(&p->prof, p->st, "pc_gj_inverse", 32.0 * cnt * msz);
        gj_launch(p, dst, cnt, n1);
      }
      if (fp32) {
        hipLaunchKernelGGL(k_to_f32, dim3(nblk(cnt * msz, 256)), dim3(256), 0, p->st, dst,
                           p->binv32 + m0 * msz, cnt * msz);
        HIPCHK(hipGetLastError());
      }
    }
    int hflag[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpyAsync(hflag, p->dflag, sizeof(int) * 4, hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    REQUIRE(hflag[0] == 0, DDA_EDEVICE, "a preconditioner block is singular");
  } catch (...) {
    if (gen) (void)hipFree(gen);
    if (scratch) (void)hipFree(scratch);
    precond_free(p);
    throw;
  }
  HIPCHK(hipFree(gen));
  if (scratch) HIPCHK(hipFree(scratch));
  p->prec_built = 1;
  p->prec_fp32 = fp32;
}

// ----------------------------------------------------------------------------- application

// One workgroup per (unique mode, chunk of rc right-hand sides).  Gathers the
// (+-wx, +-wy) mode vectors of each RHS, applies the Sx / Sy sign flips that map
// them onto the stored mode, folds into the even / odd z halves, multiplies by
// both stored inverse halves (each matrix element read once for all NV vectors,
// eight rows of both halves in flight per thread), unfolds, flips back and writes
// in place.  Workgroups are XCD-remapped so neighbouring modes share an L2.
template <typename T, int NV>
__global__ void __launch_bounds__(512) k_pc_gemv(cplx<T> *W, const cplx<T> *__restrict__ binv,
                                                 int nx, int ny, int nzw, int z0, int nz, int umx,
                                                 int hh, int n2,
                                                 int nrhs, int rc, long long nchunks, long long U,
                                                 const int *act) {
  using V = cplx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *Ub = reinterpret_cast<V *>(smem_raw);  // [2][nv][n2]
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long blk = xcd_remap(blockIdx.x, U * nchunks);
  if (blk >= U * nchunks) return;
  const long long u = blk / nchunks;
  const int r0 = (int)(blk - u * nchunks) * rc;
  const int nr = min(rc, nrhs - r0);
  if (!rhs_any_on(act, r0, nr)) return;
  const int uy = (int)(u / umx), ux = (int)(u % umx);
  const int mxs[2] = {ux, (nx - ux) % nx};
  const int mys[2] = {uy, (ny - uy) % ny};
  const int nmx = (mxs[1] != mxs[0]) ? 2 : 1;
  const int nmy = (mys[1] != mys[0]) ? 2 : 1;
  const int nmode = nmx * nmy;
  const int nv = nmode * nr;
  const long long plane = (long long)nx * ny;
  const int h = nz / 2;
  // gather + fold
  for (int e = tid; e < nv * 3 * hh; e += nt) {
    const int vi = e / (3 * hh);
    const int rem = e - vi * 3 * hh;
    const int a = rem / hh, iz = rem - a * hh;
    const int mode = vi / nr, r = r0 + vi % nr;
    const int fx = mode % nmx, fy = mode / nmx;
    const long long off = (long long)mys[fy] * nx + mxs[fx];
    const T flip = ((fx && a == 0) || (fy && a == 1)) ? (T)-1 : (T)1;
    const T sa = a == 2 ? (T)-1 : (T)1;
    const long long cb = ((long long)r * 3 + a) * nzw + z0;
    const V v1 = W[(cb + iz) * plane + off];
    const V v2 = W[(cb + (nz - 1 - iz)) * plane + off];
    Ub[vi * n2 + a * hh + iz] = cscale(cadd(v1, cscale(v2, sa)), (T)0.5 * flip);
    Ub[(nv + vi) * n2 + a * hh + iz] = cscale(csub(v1, cscale(v2, sa)), (T)0.5 * flip);
  }
  __syncthreads();
  constexpr int UNR = 8;
  const V *M0 = binv + (u * 2 + 0) * (long long)n2 * n2;
  const V *M1 = binv + (u * 2 + 1) * (long long)n2 * n2;
  const V *U0 = Ub;
  const V *U1 = Ub + (long long)nv * n2;
  for (int i0 = 0; i0 < n2; i0 += nt) {
    const int i = i0 + tid;
    const bool act = i < n2;
    V a0[NV], a1[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) { a0[v] = mk<T>((T)0, (T)0); a1[v] = mk<T>((T)0, (T)0); }
    if (act) {
      int j = 0;
      for (; j + UNR <= n2; j += UNR) {
        V m0[UNR], m1[UNR];
#pragma unroll
        for (int q = 0; q < UNR; ++q) {
          m0[q] = M0[(long long)(j + q) * n2 + i];
          m1[q] = M1[(long long)(j + q) * n2 + i];
        }
#pragma unroll
        for (int q = 0; q < UNR; ++q)
#pragma unroll
          for (int v = 0; v < NV; ++v)
            if (v < nv) {
              a0[v] = cmac(a0[v], m0[q], U0[v * n2 + j + q]);
              a1[v] = cmac(a1[v], m1[q], U1[v * n2 + j + q]);
            }
      }
      for (; j < n2; ++j) {
        const V m0 = M0[(long long)j * n2 + i], m1 = M1[(long long)j * n2 + i];
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (v < nv) {
            a0[v] = cmac(a0[v], m0, U0[v * n2 + j]);
            a1[v] = cmac(a1[v], m1, U1[v * n2 + j]);
          }
      }
    }
    // unfold + flip + scatter straight from registers: row i = (a, iz) of both halves
    if (act) {
      const int a = i / hh, iz = i - a * hh;
      const T sa = a == 2 ? (T)-1 : (T)1;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (v >= nv) continue;
        const int mode = v / nr, r = r0 + v % nr;
        const int fx = mode % nmx, fy = mode / nmx;
        const long long off = (long long)mys[fy] * nx + mxs[fx];
        const T flip = ((fx && a == 0) || (fy && a == 1)) ? (T)-1 : (T)1;
        const long long cb = ((long long)r * 3 + a) * nzw + z0;
        W[(cb + iz) * plane + off] = cscale(cadd(a0[v], a1[v]), flip);
        if (iz < h) W[(cb + (nz - 1 - iz)) * plane + off] = cscale(csub(a0[v], a1[v]), sa * flip);
      }
    }
  }
}

// One unique mode (ux, uy) of the x-y spectrum and its copies (nx - ux, ny - uy) that share
// its blocks (up to four), for the right-hand sides r0 .. r0 + nr - 1; nv = copies x nr vectors.
struct GemvMode {
  int mx0, mx1, my0, my1, nmx, nv, nr, r0;
  int nx, nzw, z0, nz, hh, n2, h;
  long long plane;
  // x-y offset of copy `mode` and the sign its flip gives component a
  __device__ __forceinline__ long long off(int mode) const {
    return (long long)(mode / nmx ? my1 : my0) * nx + (mode % nmx ? mx1 : mx0);
  }
  template <typename T> __device__ __forceinline__ T flip(int mode, int a) const {
    const int fx = mode % nmx, fy = mode / nmx;
    return ((fx && a == 0) || (fy && a == 1)) ? (T)-1 : (T)1;
  }
};

__device__ __forceinline__ GemvMode gemv_mode(long long u, int umx, int nx, int ny, int nzw, int z0,
                                              int nz, int hh, int n2, int nr, int r0) {
  GemvMode g;
  const int uy = (int)(u / umx), ux = (int)(u % umx);
  g.mx0 = ux;
  g.mx1 = (nx - ux) % nx;
  g.my0 = uy;
  g.my1 = (ny - uy) % ny;
  g.nmx = (g.mx1 != g.mx0) ? 2 : 1;
  const int nmy = (g.my1 != g.my0) ? 2 : 1;
  g.nv = g.nmx * nmy * nr;
  g.nr = nr;
  g.r0 = r0;
  g.nx = nx;
  g.nzw = nzw;
  g.z0 = z0;
  g.nz = nz;
  g.hh = hh;
  g.n2 = n2;
  g.h = nz / 2;
  g.plane = (long long)nx * ny;
  return g;
}

// Gather the mode's vectors from the y-transformed work array, flip, fold the z mirror
// halves and scale by S into Ub[2][NV][n2p] (zero beyond nv and n2).  GB elements per
// thread are loaded before any is stored.
template <typename T, int NV>
__device__ __forceinline__ void gemv_gather(cplx<T> *Ub, const cplx<T> *W, const GemvMode &g,
                                            int n2p, int tid, int nt) {
  using V = cplx<T>;
  constexpr int GB = 4;
  const int ne = NV * n2p;
  for (int e0 = 0; e0 < ne; e0 += GB * nt) {
    V v1[GB], v2[GB];
#pragma unroll
    for (int k = 0; k < GB; ++k) {
      const int e = e0 + k * nt + tid;
      const int vi = e / n2p, row = e - (e / n2p) * n2p;
      v1[k] = v2[k] = mk<T>((T)0, (T)0);
      if (e < ne && row < g.n2 && vi < g.nv) {
        const int a = row / g.hh, iz = row - a * g.hh;
        const int mode = vi / g.nr, r = g.r0 + vi % g.nr;
        const long long off = g.off(mode);
        const long long cb = ((long long)r * 3 + a) * g.nzw + g.z0;
        v1[k] = W[(cb + iz) * g.plane + off];
        v2[k] = W[(cb + (g.nz - 1 - iz)) * g.plane + off];
      }
    }
#pragma unroll
    for (int k = 0; k < GB; ++k) {
      const int e = e0 + k * nt + tid;
      if (e >= ne) continue;
      const int vi = e / n2p, row = e - (e / n2p) * n2p;
      const int a = row < g.n2 ? row / g.hh : 0;
      const T flip = g.flip<T>(vi / g.nr, a);
      const T sa = a == 2 ? (T)-1 : (T)1;
      Ub[vi * n2p + row] = cscale(cadd(v1[k], cscale(v2[k], sa)), (T)0.5 * flip * sa);
      Ub[(NV + vi) * n2p + row] = cscale(csub(v1[k], cscale(v2[k], sa)), (T)0.5 * flip * sa);
    }
  }
}

// Store one product entry: e0, e1 are the halves' values of row i in this lane's column
// (Re of vector v; the partner lane ^ 8 holds its Im).  Unfold the halves, flip, scatter to
// the row's two mirror layers.  Every lane calls it (the shuffle).
template <typename T>
__device__ __forceinline__ void gemv_store(cplx<T> *W, const GemvMode &g, T e0, T e1, int i, int v,
                                           bool im) {
  using V = cplx<T>;
  const T o0 = __shfl_xor(e0, 8, 64), o1 = __shfl_xor(e1, 8, 64);
  if (im || v >= g.nv || i >= g.n2) return;
  const V y0 = mk<T>(e0, o0), y1 = mk<T>(e1, o1);
  const int a = i / g.hh, iz = i - a * g.hh;
  const T sa = a == 2 ? (T)-1 : (T)1;
  const int mode = v / g.nr, r = g.r0 + v % g.nr;
  const long long off = g.off(mode);
  const T flip = g.flip<T>(mode, a);
  const long long cb = ((long long)r * 3 + a) * g.nzw + g.z0;
  W[(cb + iz) * g.plane + off] = cscale(cadd(y0, y1), flip);
  if (iz < g.h) W[(cb + (g.nz - 1 - iz)) * g.plane + off] = cscale(csub(y0, y1), sa * flip);
}

// Symmetric block product on the matrix cores (even nz).  One workgroup per (unique mode,
// chunk of rc <= 2 NCB right-hand sides): the up to 4 mode copies x rc vectors form an
// n2 x 8 NCB complex block U per half, and Y U is computed as the real product
// [Re Y | Im Y] x [[Re U, Im U], [-Im U, Re U]] in NCB column blocks of 16 (n2 x 2 n2 times
// 2 n2 x 16 each), with 16 x 16 x 4 MFMAs; each tile fragment feeds all NCB blocks.  Wave w
// computes tile rows I = w, w + NW, ...; step s pairs row I with J = (s - I) mod ntr, taking the
// stored tile (I, J) directly or (J, I) transposed, so the two rows that share a stored tile
// read it in the same step.  Tiles are fetched up to three steps ahead of their use.
template <typename T, int NWMAX, int NCB>
__global__ void __launch_bounds__(64 * NWMAX) k_pc_gemv_mfma(cplx<T> *W, const cplx<T> *__restrict__ pk,
                                                             int nx, int ny, int nzw, int z0, int nz,
                                                             int umx, int hh,
                                                             int n2, int ntr, int nrhs, int rc,
                                                             long long nchunks, long long U,
                                                             const int *act) {
  using V = cplx<T>;
  using v4 = typename Mfma<T>::v4;
  constexpr int NV = 8 * NCB;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *Ub = reinterpret_cast<V *>(smem_raw);  // [2][NV][n2p], zero beyond nv and n2
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long blk = xcd_remap(blockIdx.x, U * nchunks);
  if (blk >= U * nchunks) return;
  const long long u = blk / nchunks;
  const int r0 = (int)(blk - u * nchunks) * rc;
  const int nr = min(rc, nrhs - r0);
  if (!rhs_any_on(act, r0, nr)) return;
  const GemvMode g = gemv_mode(u, umx, nx, ny, nzw, z0, nz, hh, n2, nr, r0);
  const int n2p = 16 * ntr;
  gemv_gather<T, NV>(Ub, W, g, n2p, tid, nt);
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  const int r = lane & 15, q = lane >> 4;  // A: row r, k-slot q; B and D: column r
  const int vj = r & 7;
  const bool im = r >= 8;
  const long long tiles = (long long)ntr * (ntr + 1) / 2;
  for (int I = wv; I < ntr; I += nw) {
    v4 c[2][NCB];
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      const V *P = pk + (u * 2 + hf) * tiles * 256;
      const V *Uh = Ub + (hf * NV + vj) * n2p + q;  // column block cb adds 8 cb n2p
      v4 acc[NCB];
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[cb] = v4{0, 0, 0, 0};
      auto fetch = [&](int s, V (&a)[4]) {
        const int J = (s + ntr - I) % ntr;
        const long long t = J <= I ? (long long)I * (I + 1) / 2 + J : (long long)J * (J + 1) / 2 + I;
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] = P[t * 256 + (J <= I ? lane + 64 * k : tile_pos(4 * k + q, r))];
      };
      auto mac = [&](int s, const V (&a)[4]) {
        const int J = (s + ntr - I) % ntr;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
          V x[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) x[k] = Uh[8 * cb * n2p + 16 * J + 4 * k];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            acc[cb] = Mfma<T>::mma(a[k].x, im ? x[k].y : x[k].x, acc[cb]);
            acc[cb] = Mfma<T>::mma(a[k].y, im ? x[k].x : -x[k].y, acc[cb]);
          }
        }
      };
      // D - 1 tiles in flight: three; two in FP64 with one column block (measured faster);
      // one in FP64 with four column blocks and FP32 with eight (more would spill)
      constexpr int D = ((sizeof(T) == 8 && NCB >= 4) || NCB >= 8) ? 2
                        : (sizeof(T) == 8 && NCB == 1) ? 3 : 4;
      V buf[D][4];
      fetch(0, buf[0]);
#pragma unroll
      for (int d = 1; d < D - 1; ++d)
        if (d < ntr) fetch(d, buf[d]);
      for (int s = 0; s < ntr; s += D) {
#pragma unroll
        for (int b = 0; b < D; ++b) {
          if (s + b + D - 1 < ntr) fetch(s + b + D - 1, buf[(b + D - 1) % D]);
          if (s + b < ntr) mac(s + b, buf[b]);
        }
      }
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) c[hf][cb] = acc[cb];
    }
    // D[i][j] sits in column lane j, item m, row Mfma<T>::row(q, m): lane j < 8 holds Re of
    // vector j, lane j + 8 its Im.  Unfold the halves, flip, scatter.
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
      for (int m = 0; m < 4; ++m)
        gemv_store<T>(W, g, c[0][cb][m], c[1][cb][m], 16 * I + Mfma<T>::row(q, m), 8 * cb + vj, im);
  }
}

template <typename T>
static void pc_apply(dda_problem *p, int nrhs, const double2 *x, double2 *y, const cplx<T> *binv,
                     const double *xscale) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const double sz = sizeof(cplx<T>);
  cplx<T> *W = reinterpret_cast<cplx<T> *>(p->w0);
  const long long rows = (long long)nrhs * 3 * nz * ny;
  const char *suf = sizeof(T) == 8 ? "f64" : "f32";
  char nm[64];
  {
    RowArgs a{};
    a.rows = rows;
    a.n_in = nx;
    a.n_out = nx;
    a.in_stride = nx;
    a.out_stride = nx;
    a.sign = -1;
    a.cidx = p->cidx;
    a.nocc = p->nocc;
    a.vox_rows = (long long)nz * ny;
    a.rhs_rows = 3LL * nz * ny;
    a.nx = nx;
    a.N = p->N;
    a.xscale = xscale;
    snprintf(nm, sizeof nm, "pc_x_fwd_%s", suf);
    launch_rows<T, ROW_PC_FWD, double2, cplx<T>>(p, p->ux, x, W, a, nm,
                                                 rows * (4.0 * nx + sz * nx) + nrhs * 48.0 * p->nocc,
                                                 FP_PC_X_FWD);
  }
  snprintf(nm, sizeof nm, "pc_y_fwd_%s", suf);
  launch_strided<T>(p, p->uy, W, W, (long long)nrhs * 3 * nz, nx, ny, ny, (long long)ny * nx,
                    (long long)ny * nx, -1, nm, 2.0 * rows * nx * sz, 3LL * nz, FP_PC_Y_FWD);
  if (!p->tune_xy) {
    const long long U = (long long)p->umx * p->umy;
    snprintf(nm, sizeof nm, "pc_gemv_%s", suf);
    if (p->psym) {
      // right-hand sides per workgroup: 4 mode copies x rc vectors <= 8 NCB columns of U; more
      // column blocks stream each tile once for more right-hand sides, as LDS allows
      const int n2p = 16 * p->ntr;
      auto lds_of = [&](int ncb) { return (size_t)2 * 8 * ncb * n2p * sizeof(cplx<T>); };
      int ncb = nrhs <= 2 ? 1 : nrhs <= 4 ? 2 : (nrhs <= 8 || sizeof(T) == 8) ? 4 : 8;
      while (ncb > 1 && lds_of(ncb) > kLdsMax) ncb /= 2;
      const int rc = std::max(1, std::min(2 * ncb, nrhs));
      const long long nchunks = (nrhs + rc - 1) / rc;
      const size_t lds = lds_of(ncb);
      const long long tiles = (long long)p->ntr * (p->ntr + 1) / 2;
      const double bytes = (double)U * 2.0 * tiles * 256 * sz * nchunks + 2.0 * rows * nx * sz;
      const int threads = 64 * std::min(12, p->ntr);  // one wave per tile row up to 12 rows
      const dim3 grid((unsigned)xcd_grid(U * nchunks));
      KTimer t(&p->prof, p->st, nm, bytes);
      {
      auto fn = ncb == 1 ? k_pc_gemv_mfma<T, 12, 1>
                : ncb == 2 ? k_pc_gemv_mfma<T, 12, 2>
                : ncb == 4 ? k_pc_gemv_mfma<T, 12, 4>
                           : k_pc_gemv_mfma<T, 12, sizeof(T) == 8 ? 4 : 8>;
      set_lds_limit((const void *)fn, lds);
      hipLaunchKernelGGL(fn, grid, dim3(threads), lds, p->st, W, binv, nx, ny, nz, p->pz0, p->pbz,
                         p->umx, p->hh, p->n2, p->ntr, nrhs, rc, nchunks, U, p->act);
      HIPCHK(hipGetLastError());
      }
    } else {
    // right-hand sides per workgroup: up to 4 mode copies x rc vectors <= 16, LDS <= 64 KB
    int rc = std::max(1, std::min(4, nrhs));
    while (rc > 1 && (size_t)2 * 4 * rc * p->n2 * sizeof(cplx<T>) > 65536) --rc;
    const long long nchunks = (nrhs + rc - 1) / rc;
    const size_t lds = (size_t)2 * 4 * rc * p->n2 * sizeof(cplx<T>);
    int threads = ((p->n2 + 63) / 64) * 64;
    threads = std::min(512, std::max(64, threads));
    const double bytes = (double)U * 2.0 * p->n2 * p->n2 * sz * nchunks + 2.0 * rows * nx * sz;
    const int nvmax = 4 * rc;
    const dim3 grid((unsigned)xcd_grid(U * nchunks));
    KTimer t(&p->prof, p->st, nm, bytes);
    if (nvmax <= 4) {
      auto fn = k_pc_gemv<T, 4>;
      set_lds_limit((const void *)fn, lds);
      hipLaunchKernelGGL(fn, grid, dim3(threads), lds, p->st, W, binv, nx, ny, nz, p->pz0, p->pbz,
                         p->umx, p->hh, p->n2, nrhs, rc, nchunks, U, p->act);
    } else if (nvmax <= 8) {
      auto fn = k_pc_gemv<T, 8>;
      set_lds_limit((const void *)fn, lds);
      hipLaunchKernelGGL(fn, grid, dim3(threads), lds, p->st, W, binv, nx, ny, nz, p->pz0, p->pbz,
                         p->umx, p->hh, p->n2, nrhs, rc, nchunks, U, p->act);
    } else {
      auto fn = k_pc_gemv<T, 16>;
      set_lds_limit((const void *)fn, lds);
      hipLaunchKernelGGL(fn, grid, dim3(threads), lds, p->st, W, binv, nx, ny, nz, p->pz0, p->pbz,
                         p->umx, p->hh, p->n2, nrhs, rc, nchunks, U, p->act);
    }
    HIPCHK(hipGetLastError());
    }
  }
  snprintf(nm, sizeof nm, "pc_y_inv_%s", suf);
  launch_strided<T>(p, p->uy, W, W, (long long)nrhs * 3 * nz, nx, ny, ny, (long long)ny * nx,
                    (long long)ny * nx, +1, nm, 2.0 * rows * nx * sz, 3LL * nz, FP_PC_Y_INV);
  {
    RowArgs a{};
    a.rows = rows;
    a.n_in = nx;
    a.n_out = nx;
    a.in_stride = nx;
    a.out_stride = nx;
    a.sign = +1;
    a.cidx = p->cidx;
    a.nocc = p->nocc;
    a.vox_rows = (long long)nz * ny;
    a.rhs_rows = 3LL * nz * ny;
    a.nx = nx;
    a.N = p->N;
    a.scale = 1.0 / ((double)nx * ny);
    snprintf(nm, sizeof nm, "pc_x_inv_%s", suf);
    launch_rows<T, ROW_PC_INV, cplx<T>, double2>(p, p->ux, W, y, a, nm,
                                                 rows * (sz * nx + 4.0 * nx) + nrhs * 48.0 * p->nocc, FP_PC_X_INV);
  }
}

// 1-level application: one workgroup per (unique x mode u, chunk of rc right-hand sides).
// Gathers the mode copies kx = u and nx - u of each RHS (the x component negated on the copy,
// D(-w) = Sx D(w) Sx), multiplies by the stored inverse (column-major, each element read
// once for all NV vectors) and writes back in place.
template <typename T, int NV>
__global__ void __launch_bounds__(256) k_pc1_gemv(cplx<T> *W, const cplx<T> *__restrict__ binv,
                                                  int nx, int ny, int nz, int umx, int n1, int nrhs,
                                                  int rc, long long nchunks, const int *act) {
  using V = cplx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *Ub = reinterpret_cast<V *>(smem_raw);  // [nv][n1]
  const int tid = threadIdx.x, nt = blockDim.x;
  const long long blk = xcd_remap(blockIdx.x, umx * nchunks);
  if (blk >= umx * nchunks) return;
  const int u = (int)(blk / nchunks);
  const int r0 = (int)(blk - (long long)u * nchunks) * rc;
  const int nr = min(rc, nrhs - r0);
  if (!rhs_any_on(act, r0, nr)) return;
  const int kxs[2] = {u, (nx - u) % nx};
  const int nmode = kxs[1] != kxs[0] ? 2 : 1;
  const int nv = nmode * nr;
  const int m = nz * ny;
  for (int e = tid; e < nv * n1; e += nt) {
    const int vi = e / n1, i = e - vi * n1;
    const int mode = vi / nr, r = r0 + vi % nr;
    const int a = i / m, yz = i - a * m;
    V v = W[(((long long)r * 3 + a) * m + yz) * nx + kxs[mode]];
    if (mode == 1 && a == 0) v = mk<T>(-v.x, -v.y);
    Ub[e] = v;
  }
  __syncthreads();
  const V *M = binv + (long long)u * n1 * n1;
  constexpr int UNR = 4;
  for (int i = tid; i < n1; i += nt) {
    V acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = mk<T>((T)0, (T)0);
    int j = 0;
    for (; j + UNR <= n1; j += UNR) {
      V mv[UNR];
#pragma unroll
      for (int q = 0; q < UNR; ++q) mv[q] = M[(long long)(j + q) * n1 + i];
#pragma unroll
      for (int q = 0; q < UNR; ++q)
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (v < nv) acc[v] = cmac(acc[v], mv[q], Ub[v * n1 + j + q]);
    }
    for (; j < n1; ++j) {
      const V mv = M[(long long)j * n1 + i];
#pragma unroll
      for (int v = 0; v < NV; ++v)
        if (v < nv) acc[v] = cmac(acc[v], mv, Ub[v * n1 + j]);
    }
    const int a = i / m, yz = i - a * m;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      if (v >= nv) continue;
      const int mode = v / nr, r = r0 + v % nr;
      V y = acc[v];
      if (mode == 1 && a == 0) y = mk<T>(-y.x, -y.y);
      W[(((long long)r * 3 + a) * m + yz) * nx + kxs[mode]] = y;
    }
  }
}

template <typename T>
static void pc_apply1(dda_problem *p, int nrhs, const double2 *x, double2 *y, const cplx<T> *binv,
                      const double *xscale) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const double sz = sizeof(cplx<T>);
  cplx<T> *W = reinterpret_cast<cplx<T> *>(p->w0);
  const long long rows = (long long)nrhs * 3 * nz * ny;
  const char *suf = sizeof(T) == 8 ? "f64" : "f32";
  char nm[64];
  RowArgs a{};
  a.rows = rows;
  a.n_in = nx;
  a.n_out = nx;
  a.in_stride = nx;
  a.out_stride = nx;
  a.cidx = p->cidx;
  a.nocc = p->nocc;
  a.vox_rows = (long long)nz * ny;
  a.rhs_rows = 3LL * nz * ny;
  a.nx = nx;
  a.N = p->N;
  {
    RowArgs f = a;
    f.sign = -1;
    f.xscale = xscale;
    snprintf(nm, sizeof nm, "pc_x_fwd_%s", suf);
    launch_rows<T, ROW_PC_FWD, double2, cplx<T>>(p, p->ux, x, W, f, nm,
                                                 rows * (4.0 * nx + sz * nx) + nrhs * 48.0 * p->nocc);
  }
  {
    const int n1 = p->n2;
    const int rc = std::max(1, std::min(2, nrhs));
    const long long nchunks = (nrhs + rc - 1) / rc;
    const size_t lds = (size_t)2 * rc * n1 * sizeof(cplx<T>);
    const int threads = std::min(256, ((n1 + 63) / 64) * 64);
    const double bytes = (double)p->umx * n1 * n1 * sz * nchunks + 2.0 * rows * nx * sz;
    snprintf(nm, sizeof nm, "pc1_gemv_%s", suf);
    KTimer t(&p->prof, p->st, nm, bytes);
    auto fn = k_pc1_gemv<T, 4>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)xcd_grid((long long)p->umx * nchunks)), dim3(threads), lds,
                       p->st, W, binv, nx, ny, nz, p->umx, n1, nrhs, rc, nchunks, p->act);
    HIPCHK(hipGetLastError());
  }
  {
    RowArgs b = a;
    b.sign = +1;
    b.scale = 1.0 / (double)nx;
    snprintf(nm, sizeof nm, "pc_x_inv_%s", suf);
    launch_rows<T, ROW_PC_INV, cplx<T>, double2>(p, p->ux, W, y, b, nm,
                                                 rows * (sz * nx + 4.0 * nx) + nrhs * 48.0 * p->nocc);
  }
}

// Q: the circulant preconditioner as applied, occupied voxels in and out
static void apply_circulant(dda_problem *p, int nrhs, const double2 *x, double2 *y, int fp32,
                            const double *xscale) {
  if (p->opt.precond == 1) {
    if (fp32)
      pc_apply1<float>(p, nrhs, x, y, p->binv32, xscale);
    else
      pc_apply1<double>(p, nrhs, x, y, p->binv64, xscale);
  } else if (fp32) {
    pc_apply<float>(p, nrhs, x, y, p->binv32, xscale);
  } else {
    pc_apply<double>(p, nrhs, x, y, p->binv64, xscale);
  }
}

void apply_precond(dda_problem *p, int nrhs, const double2 *x, double2 *y, int fp32,
                   const double *xscale) {
  REQUIRE(p->prec_built, DDA_ESTATE, "preconditioner not built");
  REQUIRE(fp32 == p->prec_fp32, DDA_ESTATE, "preconditioner was built in %s",
          p->prec_fp32 ? "FP32" : "FP64");
  const int k = p->opt.diag_steps;
  if (k <= 0) {
    apply_circulant(p, nrhs, x, y, fp32, xscale);
    return;
  }
  // circulant-plus-diagonal P = D + C = B + Delta (Sec. 1, Sec. 5): z_0 = Q v,
  // z_{i+1} = Q (v - Delta z_i), v = s x.  x is read by every step, so an in-place call keeps
  // z in pdz until the last step writes y.
  double2 *z = x == y ? p->pdz : y;
  apply_circulant(p, nrhs, x, z, fp32, xscale);
  for (int i = 1; i <= k; ++i) {
    {
      KTimer t(&p->prof, p->st, "pc_diag_resid", (48.0 * 3 * nrhs + 16.0) * p->nocc);
      hipLaunchKernelGGL(k_diag_resid, dim3(nblk(p->nocc, 256), 3 * nrhs), dim3(256), 0, p->st, x,
                         z, p->pdelta, p->pdt, p->nocc, xscale, p->act);
      HIPCHK(hipGetLastError());
    }
    apply_circulant(p, nrhs, p->pdt, i == k ? y : z, fp32, nullptr);
  }
}

}  // namespace dda
