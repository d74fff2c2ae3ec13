// Fused z pass (z-FFT, 3x3 multiply by the kernel spectrum, inverse z-FFT) with the
// transforms held in registers, for FFT lengths n = 2 nz = G * P that are powers of two
// with P = G or P = 2G (n = 32 .. 256).
//
// Each (column, component) is transformed by G threads.  Forward: thread g holds the
// samples x[g + G b] (b < P, only b < P/2 non-zero because the upper half of the padded
// column is zero), does a P-point DFT over b in registers, twiddles by W_n^{g c}, and one
// LDS exchange hands thread g the columns c = g + G j of the G x P array, which it
// transforms over g with G-point DFTs.  The spectrum value at frequency k = g + G b then
// sits in thread g for every component, so the 3x3 product needs one exchange across the
// three component groups of a column.  The inverse transform starts from exactly that
// ownership (input index g + G b), so it needs one more exchange and no other permutation;
// only the first nz outputs are formed and stored.  Three LDS exchanges in all, against two
// per radix pass for a transform staged entirely in LDS.  Each exchange moves real and
// imaginary parts (or two halves of the frequencies) in turn, which halves its LDS, and the
// workgroup's slab of kernel spectrum is staged in LDS with coalesced loads issued together
// with the field loads, so the 3x3 product never waits on global memory.
//
// Work assignment: a workgroup takes TW consecutive octant columns (ox, oy) of the kernel
// spectrum in one of the four sign mirrors (kx = ox or 2 nx - ox, ky = oy or 2 ny - oy) for
// one right-hand side, all three components.  The logical block index runs fastest over
// RHS and mirrors, so the 4 R workgroups that read the same kernel-spectrum columns are
// adjacent and, through the XCD remap, share one L2.  The kernel spectrum is stored z-major,
// [oy][ox][oz][6], so a workgroup's slab is one contiguous range.
#pragma once

#include "fft_engine.h"

namespace dda {

// cos(pi j / 16), j in [0, 8]
__host__ __device__ constexpr double qcos16(int j) {
  return j == 0   ? 1.0
         : j == 1 ? 0.98078528040323044912
         : j == 2 ? 0.92387953251128675613
         : j == 3 ? 0.83146961230254523708
         : j == 4 ? 0.70710678118654752440
         : j == 5 ? 0.55557023301960222474
         : j == 6 ? 0.38268343236508977173
         : j == 7 ? 0.19509032201612826785
                  : 0.0;
}
// cos and sin of 2 pi k / 32
__host__ __device__ constexpr double root32_cos(int k) {
  k &= 31;
  return k <= 8 ? qcos16(k) : k < 16 ? -qcos16(16 - k) : k <= 24 ? -qcos16(k - 16) : qcos16(32 - k);
}
__host__ __device__ constexpr double root32_sin(int k) { return root32_cos((k + 24) & 31); }

// a * exp(SIGN 2 pi i k / 32), exact for multiples of a quarter turn
template <int SIGN, typename V> __device__ __forceinline__ V rot32(V a, int k) {
  using T = typename RealOf<V>::type;
  k &= 31;
  if (k == 0) return a;
  if (k == 16) return mk<T>(-a.x, -a.y);
  if (k == 8) return cmuli(a, SIGN);
  if (k == 24) return cmuli(a, -SIGN);
  return cmul(a, mk<T>((T)root32_cos(k), (T)(SIGN * root32_sin(k))));
}

// N-point DFT in registers, N in {2, 4, 8, 16, 32}; SIGN = -1 forward, +1 inverse.
template <int N, int SIGN, typename V> __device__ __forceinline__ void rdft(V *a) {
  if constexpr (N <= 8) {
    dft<N, V>(a, SIGN);
  } else {
    constexpr int H = N / 2;
    V e[H], o[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      e[i] = a[2 * i];
      o[i] = a[2 * i + 1];
    }
    rdft<H, SIGN, V>(e);
    rdft<H, SIGN, V>(o);
#pragma unroll
    for (int c = 0; c < H; ++c) {
      const V t = rot32<SIGN>(o[c], c * (32 / N));
      a[c] = cadd(e[c], t);
      a[c + H] = csub(e[c], t);
    }
  }
}

// N-point DFT of x[0 .. N/2) padded with N/2 zeros: X[2c] and X[2c + 1] are the N/2-point
// DFTs of x[b] and x[b] W_N^b.
template <int N, int SIGN, typename V> __device__ __forceinline__ void rdft_half(const V *x, V *X) {
  constexpr int H = N / 2;
  V e[H], o[H];
#pragma unroll
  for (int b = 0; b < H; ++b) {
    e[b] = x[b];
    o[b] = rot32<SIGN>(x[b], b * (32 / N));
  }
  rdft<H, SIGN, V>(e);
  rdft<H, SIGN, V>(o);
#pragma unroll
  for (int c = 0; c < H; ++c) {
    X[2 * c] = e[c];
    X[2 * c + 1] = o[c];
  }
}

struct ZRArgs {
  int nx, ny, nz;     // grid; the transform length is 2 nz
  long long plane;    // elements between z rows of the work array (>= 4 nx ny)
  int tw;             // octant columns per workgroup (power of two)
  int tiles_x;        // ceil((nx + 1) / tw)
  int nrhs;
  long long nblk;     // (ny + 1) tiles_x 4 nrhs, RHS fastest, then mirror, then tile
};

// Position of element (row, c) of a G x P exchange tile: XOR-swizzled so that both the
// row-wise writes and the column-wise reads of 16 lanes fall in distinct LDS banks.
template <int P> __device__ __forceinline__ int zr_at(int row, int c) {
  return row * P + (c ^ (row & (P - 1)));
}

template <typename T, int G, int P>
__global__ void __launch_bounds__(256) k_zpass_reg(cplx<T> *data, const cplx<T> *__restrict__ tw,
                                                   const cplx<T> *__restrict__ khat, ZRArgs a) {
  using V = cplx<T>;
  constexpr int n = G * P, M = P / G, HB = P / 2;
  static_assert(M == 1 || M == 2, "P must be G or 2G");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *s = reinterpret_cast<V *>(smem_raw);
  const long long blk = xcd_remap(blockIdx.x, a.nblk);
  if (blk >= a.nblk) return;
  const int r = (int)(blk % a.nrhs);
  long long q = blk / a.nrhs;
  const int mir = (int)(q & 3);
  q >>= 2;
  const int tx = (int)(q % a.tiles_x);
  const int oy = (int)(q / a.tiles_x);
  if ((mir & 2) && (oy == 0 || oy == a.ny)) return;  // ky mirror of a self-mirrored row
  const int g = threadIdx.x & (G - 1);
  const int col = (threadIdx.x / G) & (a.tw - 1);
  const int comp = threadIdx.x / (G * a.tw);
  const int ox = tx * a.tw + col;
  const bool ok = ox <= a.nx && !((mir & 1) && (ox == 0 || ox == a.nx));
  const int kx = (mir & 1) ? 2 * a.nx - ox : ox;
  const int ky = (mir & 2) ? 2 * a.ny - oy : oy;
  V *cb = data + ((long long)r * 3 + comp) * a.nz * a.plane + (long long)ky * 2 * a.nx + kx;
  // LDS: exchange region (3 tw tiles of n reals, or of G x P/2 complex), twiddles, and the
  // kernel-spectrum slab of the workgroup's octant columns, [tw][nz+1][6]
  T *exd = reinterpret_cast<T *>(s);
  V *exc = s;
  V *stw = reinterpret_cast<V *>(reinterpret_cast<unsigned char *>(s) + (size_t)3 * a.tw * n * sizeof(T));
  V *kh = stw + n;
  const int tile = comp * a.tw + col;
  T *ed = exd + tile * n;
  constexpr int PH = P / 2;

  // issue the field loads first, then the spectrum slab (coalesced) and the twiddles
  V x[HB];
#pragma unroll
  for (int b = 0; b < HB; ++b)
    x[b] = ok ? cb[(long long)(g + G * b) * a.plane] : mk<T>((T)0, (T)0);
  {
    const int nval = min(a.tw, a.nx + 1 - tx * a.tw);  // >= 1: tx * tw <= nx
    const long long slab = (long long)nval * (a.nz + 1) * 6;
    const V *src = khat + ((long long)oy * (a.nx + 1) + (long long)tx * a.tw) * (a.nz + 1) * 6;
    constexpr int KB = 16;
    for (long long e0 = threadIdx.x; e0 < slab; e0 += (long long)KB * blockDim.x) {
      V t[KB];
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        const long long e = e0 + (long long)i * blockDim.x;
        t[i] = e < slab ? src[e] : mk<T>((T)0, (T)0);
      }
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        const long long e = e0 + (long long)i * blockDim.x;
        if (e < slab) kh[e] = t[i];
      }
    }
    for (int t = threadIdx.x; t < n; t += blockDim.x) stw[t] = tw[t];
  }
  __syncthreads();

  // forward: P-point DFTs over b of the non-zero half, twiddle
  V X[P];
  rdft_half<P, -1, V>(x, X);
#pragma unroll
  for (int c = 1; c < P; ++c) X[c] = cmul(X[c], stw[g * c]);
  // exchange (real parts, then imaginary parts) and G-point DFTs over the rows; frequency
  // g + G b lands in X[b]
  V Y[P];
#pragma unroll
  for (int c = 0; c < P; ++c) ed[zr_at<P>(g, c)] = X[c].x;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int a_ = 0; a_ < G; ++a_) Y[j * G + a_].x = ed[zr_at<P>(a_, g + G * j)];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < P; ++c) ed[zr_at<P>(g, c)] = X[c].y;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int a_ = 0; a_ < G; ++a_) Y[j * G + a_].y = ed[zr_at<P>(a_, g + G * j)];
#pragma unroll
  for (int j = 0; j < M; ++j) {
    rdft<G, -1, V>(Y + j * G);
#pragma unroll
    for (int d = 0; d < G; ++d) X[j + M * d] = Y[j * G + d];
  }

  // 3x3 product with the kernel spectrum, in two halves of this thread's frequencies: publish
  // this component's half, read the other two components' values and the spectrum from LDS
  {
    const int c1 = comp == 0 ? 1 : 0, c2 = comp == 2 ? 1 : 2;  // the other two components
    const V *s1 = exc + (c1 * a.tw + col) * G * PH, *s2 = exc + (c2 * a.tw + col) * G * PH;
    V *so = exc + tile * G * PH;
    const int k_own = comp_index(comp, comp), k_1 = comp_index(comp, c1), k_2 = comp_index(comp, c2);
    const V *kc = kh + (ok ? col : 0) * (a.nz + 1) * 6;
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < PH; ++i) so[g * PH + (i ^ (g & (PH - 1)))] = X[hf * PH + i];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < PH; ++i) {
        const int b = hf * PH + i;
        const int k = g + G * b;
        const int oz = k <= a.nz ? k : n - k;
        const int mr = (mir & 3) | (k > a.nz ? 4 : 0);
        const V *K = kc + oz * 6;
        V k0 = K[k_own], k1 = K[k_1], k2 = K[k_2];
        if (__popc(comp_odd_mask(k_own) & mr) & 1) k0 = mk<T>(-k0.x, -k0.y);
        if (__popc(comp_odd_mask(k_1) & mr) & 1) k1 = mk<T>(-k1.x, -k1.y);
        if (__popc(comp_odd_mask(k_2) & mr) & 1) k2 = mk<T>(-k2.x, -k2.y);
        const int e = g * PH + (i ^ (g & (PH - 1)));
        X[b] = cadd(cadd(cmul(k0, X[b]), cmul(k1, s1[e])), cmul(k2, s2[e]));
      }
    }
  }

  // inverse: P-point DFTs over b (input index g + G b), twiddle, exchange as above
  rdft<P, +1, V>(X);
#pragma unroll
  for (int c = 1; c < P; ++c) X[c] = cmulcj(stw[g * c], X[c]);
  __syncthreads();
#pragma unroll
  for (int c = 0; c < P; ++c) ed[zr_at<P>(g, c)] = X[c].x;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int a_ = 0; a_ < G; ++a_) Y[j * G + a_].x = ed[zr_at<P>(a_, g + G * j)];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < P; ++c) ed[zr_at<P>(g, c)] = X[c].y;
  __syncthreads();
#pragma unroll
  for (int j = 0; j < M; ++j)
#pragma unroll
    for (int a_ = 0; a_ < G; ++a_) Y[j * G + a_].y = ed[zr_at<P>(a_, g + G * j)];
  // G-point DFTs over the rows, first half of the outputs only (rows c + P d < nz)
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int c = g + G * j;
    rdft<G, +1, V>(Y + j * G);
    if (ok) {
#pragma unroll
      for (int d = 0; d < G / 2; ++d) cb[(long long)(c + P * d) * a.plane] = Y[j * G + d];
    }
  }
}

}  // namespace dda
