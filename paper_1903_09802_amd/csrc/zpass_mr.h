// Fused z pass (z-FFT, 3x3 multiply by the kernel spectrum, inverse z-FFT) with the
// transforms held in registers, for FFT lengths n = 2 nz = G P with G and P even, built from
// the radices 2, 3, 5 and 7 (powers of two included).
//
// The length-n transform is split as n = G x P.  Forward: thread g < G holds the samples
// x[g + G b] (only b < P/2 are non-zero: the padded upper half of the column is zero), takes
// the P-point DFT over b in registers and twiddles by W_n^{g c}; one LDS exchange gives
// thread c < P the values of every g, and its G-point DFT over g leaves the spectrum at the
// frequencies k = c + P d (d < G) in thread c.  When P = M G (M > 1) the G threads of a
// column each take M of the frequency columns, c = t + G j, so no thread idles; otherwise
// (P <= G) a column has G threads of which the first P hold frequencies.  The 3x3 product
// with the kernel spectrum then needs one exchange across the three component groups of a
// column.  The inverse runs the
// same split transposed: thread c takes the G-point inverse DFT over d and twiddles by
// conj W_n^{c e}; after one exchange thread e < G takes the P-point inverse DFT over c,
// giving the outputs e + G f, of which f < P/2 (the first nz) are stored back to the rows
// the forward loaded.  The DFTs of composite length
// are Cooley-Tukey splits down to the radices 2..8 with compile-time twiddles.  Each exchange
// moves real and imaginary parts (or two halves of the frequencies) in turn, which halves
// its LDS.
//
// Work assignment: an item is one of the four sign mirrors (kx = ox or 2 nx - ox, ky = oy or
// 2 ny - oy) of TW consecutive octant columns (ox, oy) for one right-hand side, all three
// components.  The 4 R items of a tile share its kernel-spectrum slab ([oy][ox][oz][6], one
// contiguous range, staged once in LDS); a workgroup takes IPW consecutive items of a tile
// (RHS fastest, then mirror) and issues the next item's field loads before it transforms the
// current one, so they are in flight across its arithmetic.  Barriers inside the loop order
// LDS only (a full barrier would wait for those loads).
#pragma once

#include <type_traits>

#include "fft_engine.h"

namespace dda {

// ---------------------------------------------------------------- compile-time roots of unity

constexpr double cx_pi = 3.14159265358979323846;
constexpr double cx_series_cos(double x) {  // |x| <= pi / 4
  double s = 1.0, t = 1.0;
  for (int i = 1; i <= 12; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
constexpr double cx_series_sin(double x) {  // |x| <= pi / 4
  double s = x, t = x;
  for (int i = 1; i <= 12; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double cx_sin2pi(long long m, long long N);
// cos(2 pi m / N): reflections bring the angle into [0, pi / 4], then a Taylor series
constexpr double cx_cos2pi(long long m, long long N) {
  m %= N;
  if (m < 0) m += N;
  if (2 * m > N) m = N - m;                            // cos(2 pi - t) = cos t
  if (4 * m > N) return -cx_cos2pi(N - 2 * m, 2 * N);  // cos t = -cos(pi - t)
  if (8 * m > N) return cx_sin2pi(N - 4 * m, 4 * N);   // cos t = sin(pi / 2 - t)
  return cx_series_cos(2.0 * cx_pi * (double)m / (double)N);
}
// sin(2 pi m / N)
constexpr double cx_sin2pi(long long m, long long N) {
  m %= N;
  if (m < 0) m += N;
  if (2 * m > N) return -cx_sin2pi(N - m, N);         // sin(2 pi - t) = -sin t
  if (4 * m > N) return cx_sin2pi(N - 2 * m, 2 * N);  // sin t = sin(pi - t)
  if (8 * m > N) return cx_cos2pi(N - 4 * m, 4 * N);  // sin t = cos(pi / 2 - t)
  return cx_series_sin(2.0 * cx_pi * (double)m / (double)N);
}

// a * exp(SIGN 2 pi i M / N) with M, N known at compile time; quarter turns are exact
template <int SIGN, int M, int N, typename V> __device__ __forceinline__ V twc(V a) {
  using T = typename RealOf<V>::type;
  constexpr int m = ((M % N) + N) % N;
  if constexpr (m == 0) {
    return a;
  } else if constexpr (2 * m == N) {
    return mk<T>(-a.x, -a.y);
  } else if constexpr (4 * m == N) {
    return cmuli(a, SIGN);
  } else if constexpr (4 * m == 3 * N) {
    return cmuli(a, -SIGN);
  } else {
    constexpr double c = cx_cos2pi(m, N), s = cx_sin2pi(m, N);
    return cmul(a, mk<T>((T)c, (T)(SIGN * s)));
  }
}

// f(integral_constant<int, i>) for i = I .. N-1
template <int I, int N, typename F> __device__ __forceinline__ void sfor(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    sfor<I + 1, N>(f);
  }
}

constexpr int mr_first_radix(int N) {
  return N % 4 == 0 ? 4 : N % 2 == 0 ? 2 : N % 3 == 0 ? 3 : N % 5 == 0 ? 5 : 7;
}

// N-point DFT in registers (N with factors 2, 3, 5, 7); SIGN = -1 forward, +1 inverse.
// N = N1 N2: N1-point DFTs over n1 of x[N2 n1 + n2], twiddle W_N^{n2 k1}, N2-point DFTs over
// n2, result X[k1 + N1 k2].
template <int N, int SIGN, typename V> __device__ __forceinline__ void mdft(V *a) {
  if constexpr (N == 1) {
  } else if constexpr (N == 2 || N == 3 || N == 4 || N == 5 || N == 7 || N == 8) {
    dft<N, V>(a, SIGN);
  } else {
    constexpr int N1 = mr_first_radix(N), N2 = N / N1;
    V t[N];
    sfor<0, N2>([&](auto I2) {
      constexpr int n2 = decltype(I2)::value;
      V u[N1];
#pragma unroll
      for (int n1 = 0; n1 < N1; ++n1) u[n1] = a[N2 * n1 + n2];
      dft<N1, V>(u, SIGN);
      sfor<0, N1>([&](auto I1) {
        constexpr int k1 = decltype(I1)::value;
        t[n2 * N1 + k1] = twc<SIGN, n2 * k1, N>(u[k1]);
      });
    });
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) {
      V u[N2];
#pragma unroll
      for (int n2 = 0; n2 < N2; ++n2) u[n2] = t[n2 * N1 + k1];
      mdft<N2, SIGN, V>(u);
#pragma unroll
      for (int k2 = 0; k2 < N2; ++k2) a[k1 + N1 * k2] = u[k2];
    }
  }
}

// N-point DFT (N even) of x[0 .. N/2) followed by N/2 zeros: X[2c] and X[2c + 1] are the
// N/2-point DFTs of x[b] and of x[b] W_N^b.
template <int N, int SIGN, typename V> __device__ __forceinline__ void mdft_half(const V *x, V *X) {
  constexpr int H = N / 2;
  V e[H], o[H];
  sfor<0, H>([&](auto I) {
    constexpr int b = decltype(I)::value;
    e[b] = x[b];
    o[b] = twc<SIGN, b, N>(x[b]);
  });
  mdft<H, SIGN, V>(e);
  mdft<H, SIGN, V>(o);
#pragma unroll
  for (int c = 0; c < H; ++c) {
    X[2 * c] = e[c];
    X[2 * c + 1] = o[c];
  }
}

// Frequency columns per thread (M = P / G when P is a multiple M > 1 of G, else 1), threads
// per column, and LDS bytes of a workgroup with `tw` columns: exchange tiles of G x (P + 1)
// reals (the product's exchange reuses them), the twiddles and the spectrum slab.
__host__ __device__ constexpr int zmr_ncol(int G, int P) { return P > G && P % G == 0 ? P / G : 1; }
__host__ __device__ constexpr int zmr_tpc(int G, int P) { return zmr_ncol(G, P) > 1 ? G : G > P ? G : P; }
template <typename T> inline size_t zmr_lds(int G, int P, int tw, int nz) {
  return (size_t)3 * tw * G * (P + 1) * sizeof(T) + (size_t)G * P * sizeof(cplx<T>) +
         (size_t)tw * (nz + 1) * 6 * sizeof(cplx<T>);
}

struct ZRArgs {
  int nx, ny, nz;     // grid; the transform length is 2 nz
  long long plane;    // elements between z rows of the work array (>= 4 nx ny)
  int tw;             // octant columns per item (power of two)
  int tiles_x;        // ceil((nx + 1) / tw)
  int nrhs;
  int ipw;            // items per workgroup (>= 1)
  int nch;            // workgroups per tile, ceil(4 nrhs / ipw)
  long long nblk;     // (ny + 1) tiles_x nch, chunk fastest
  const int *act;     // null, or per-right-hand-side flags: items of a right-hand side whose
                      // flag is 0 are skipped (inside a solver cycle, the ones that stopped)
};

template <typename T, int G, int P>
__global__ void __launch_bounds__(256) k_zpass_mr(cplx<T> *data, const cplx<T> *__restrict__ tw,
                                                  const cplx<T> *__restrict__ khat, ZRArgs a) {
  using V = cplx<T>;
  constexpr int n = G * P, TPC = zmr_tpc(G, P), NC = zmr_ncol(G, P), LD = P + 1, GH = G / 2,
                PH = P / 2;
  static_assert(G % 2 == 0 && P % 2 == 0, "G and P must be even");
  static_assert(NC > 1 || P <= G, "P must be at most G or a multiple of it");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const long long blk = xcd_remap(blockIdx.x, a.nblk);
  if (blk >= a.nblk) return;
  const int ch = (int)(blk % a.nch);
  const long long tb = blk / a.nch;
  const int tx = (int)(tb % a.tiles_x);
  const int oy = (int)(tb / a.tiles_x);
  // items of this tile: RHS fastest, then mirror; rows oy = 0, ny have no distinct ky mirror
  const int it0 = ch * a.ipw;
  const int it1 = min(((oy == 0 || oy == a.ny) ? 2 : 4) * a.nrhs, it0 + a.ipw);
  if (it0 >= it1) return;
  auto item_on = [&](int it) { return !a.act || a.act[it % a.nrhs] != 0; };
  {
    bool any = false;
    for (int it = it0; it < it1; ++it) any = any || item_on(it);
    if (!any) return;
  }
  const int t = (int)threadIdx.x % TPC;
  const int col = ((int)threadIdx.x / TPC) & (a.tw - 1);
  const int comp = (int)threadIdx.x / (TPC * a.tw);
  const int ox = tx * a.tw + col;
  T *exd = reinterpret_cast<T *>(smem_raw);
  V *stw = reinterpret_cast<V *>(smem_raw + (size_t)3 * a.tw * G * LD * sizeof(T));
  V *kh = stw + n;
  T *ed = exd + (comp * a.tw + col) * G * LD;
  // Thread t is sample row g = t of the forward's first and the inverse's last stage when
  // t < G, and holds the frequency columns c = t + G j (j < NC; frequencies c + P d) when
  // t < P.  Where t is out of a stage's range it takes index 0 there and so replays, bit for
  // bit, the work of thread 0 of its column: its LDS writes repeat thread 0's values at
  // thread 0's addresses, which keeps every write unconditional (a branch around them costs
  // registers); only the final global stores are masked.
  const int g = t < G ? t : 0, c = t < P ? t : 0;
  auto column = [&](int it, bool &ok) -> V * {
    const int mir = it / a.nrhs, r = it - mir * a.nrhs;
    ok = ox <= a.nx && !((mir & 1) && (ox == 0 || ox == a.nx));
    const int kx = (mir & 1) ? 2 * a.nx - ox : ox;
    const int ky = (mir & 2) ? 2 * a.ny - oy : oy;
    return data + ((long long)r * 3 + comp) * a.nz * a.plane + (long long)ky * 2 * a.nx + kx;
  };
  auto load = [&](int it, V (&x)[PH]) {
    bool ok;
    const V *cb = column(it, ok);
    ok = ok && item_on(it);
#pragma unroll
    for (int b = 0; b < PH; ++b) x[b] = ok ? cb[(long long)(g + G * b) * a.plane] : mk<T>((T)0, (T)0);
  };

  // the first item's field loads, then the spectrum slab (coalesced) and the twiddles
  V x[PH], xn[PH];
  load(it0, x);
  {
    const int nval = min(a.tw, a.nx + 1 - tx * a.tw);  // >= 1: tx * tw <= nx
    const long long slab = (long long)nval * (a.nz + 1) * 6;
    const V *src = khat + ((long long)oy * (a.nx + 1) + (long long)tx * a.tw) * (a.nz + 1) * 6;
    constexpr int KB = 16;
    for (long long e0 = threadIdx.x; e0 < slab; e0 += (long long)KB * blockDim.x) {
      V tt[KB];
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        const long long e = e0 + (long long)i * blockDim.x;
        tt[i] = e < slab ? src[e] : mk<T>((T)0, (T)0);
      }
#pragma unroll
      for (int i = 0; i < KB; ++i) {
        const long long e = e0 + (long long)i * blockDim.x;
        if (e < slab) kh[e] = tt[i];
      }
    }
    for (int i = threadIdx.x; i < n; i += blockDim.x) stw[i] = tw[i];
  }
  __syncthreads();

  for (int it = it0; it < it1; ++it) {
    if (it + 1 < it1) load(it + 1, xn);  // next item's column, in flight during this one
    if (!item_on(it)) {                  // uniform over the workgroup: no LDS use, no barrier
#pragma unroll
      for (int b = 0; b < PH; ++b) x[b] = xn[b];
      continue;
    }
    if (it > it0) lds_barrier();          // the previous item's last exchange reads are done
    const int mir = it / a.nrhs;
    bool ok;
    V *cb = column(it, ok);

    // forward stage 1: P-point DFT over b of the non-zero half, twiddle W_n^{g j}
    V X[P];
    mdft_half<P, -1, V>(x, X);
#pragma unroll
    for (int j = 1; j < P; ++j) X[j] = cmul(X[j], stw[g * j]);
    // exchange, real parts then imaginary parts: element (g, j) at ed[g LD + j]
    V Y[NC * G];
#pragma unroll
    for (int j = 0; j < P; ++j) ed[g * LD + j] = X[j].x;
    lds_barrier();
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int i = 0; i < G; ++i) Y[m * G + i].x = ed[i * LD + c + G * m];
    lds_barrier();
#pragma unroll
    for (int j = 0; j < P; ++j) ed[g * LD + j] = X[j].y;
    lds_barrier();
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int i = 0; i < G; ++i) Y[m * G + i].y = ed[i * LD + c + G * m];
    // forward stage 2: G-point DFTs over g; frequency c + G m + P d lands in Y[m G + d]
#pragma unroll
    for (int m = 0; m < NC; ++m) mdft<G, -1, V>(Y + m * G);

    // 3x3 product with the kernel spectrum in two halves of d: publish this component's
    // half, read the other two components' values at the same frequencies
    {
      const int c1 = comp == 0 ? 1 : 0, c2 = comp == 2 ? 1 : 2;
      V *so = reinterpret_cast<V *>(ed);
      const V *s1 = reinterpret_cast<const V *>(exd + (c1 * a.tw + col) * G * LD);
      const V *s2 = reinterpret_cast<const V *>(exd + (c2 * a.tw + col) * G * LD);
      const int k_own = comp_index(comp, comp), k_1 = comp_index(comp, c1), k_2 = comp_index(comp, c2);
      const V *kc = kh + (ok ? col : 0) * (a.nz + 1) * 6;
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        lds_barrier();
#pragma unroll
        for (int m = 0; m < NC; ++m)
#pragma unroll
          for (int i = 0; i < GH; ++i) so[i * P + c + G * m] = Y[m * G + hf * GH + i];
        lds_barrier();
#pragma unroll
        for (int m = 0; m < NC; ++m)
#pragma unroll
        for (int i = 0; i < GH; ++i) {
          const int d = hf * GH + i;
          const int k = c + G * m + P * d;
          const int oz = k <= a.nz ? k : n - k;
          const int mr = (mir & 3) | (k > a.nz ? 4 : 0);
          const V *K = kc + oz * 6;
          V k0 = K[k_own], k1 = K[k_1], k2 = K[k_2];
          if (__popc(comp_odd_mask(k_own) & mr) & 1) k0 = mk<T>(-k0.x, -k0.y);
          if (__popc(comp_odd_mask(k_1) & mr) & 1) k1 = mk<T>(-k1.x, -k1.y);
          if (__popc(comp_odd_mask(k_2) & mr) & 1) k2 = mk<T>(-k2.x, -k2.y);
          const int e = i * P + c + G * m;
          Y[m * G + d] = cadd(cadd(cmul(k0, Y[m * G + d]), cmul(k1, s1[e])), cmul(k2, s2[e]));
        }
      }
    }

    // inverse stage 1: G-point DFTs over d, twiddle conj W_n^{c e} (c = t + G m)
#pragma unroll
    for (int m = 0; m < NC; ++m) {
      mdft<G, +1, V>(Y + m * G);
#pragma unroll
      for (int e = 1; e < G; ++e) Y[m * G + e] = cmulcj(stw[(c + G * m) * e], Y[m * G + e]);
    }
    // exchange: element (e, c) at ed[e LD + c]
    lds_barrier();
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int e = 0; e < G; ++e) ed[e * LD + c + G * m] = Y[m * G + e].x;
    lds_barrier();
#pragma unroll
    for (int j = 0; j < P; ++j) X[j].x = ed[g * LD + j];
    lds_barrier();
#pragma unroll
    for (int m = 0; m < NC; ++m)
#pragma unroll
      for (int e = 0; e < G; ++e) ed[e * LD + c + G * m] = Y[m * G + e].y;
    lds_barrier();
#pragma unroll
    for (int j = 0; j < P; ++j) X[j].y = ed[g * LD + j];
    // inverse stage 2: P-point DFT over c; outputs g + G f, the first nz (f < P/2) are stored
    mdft<P, +1, V>(X);
    if (ok && t < G) {
#pragma unroll
      for (int f = 0; f < PH; ++f) cb[(long long)(g + G * f) * a.plane] = X[f];
    }
#pragma unroll
    for (int b = 0; b < PH; ++b) x[b] = xn[b];
  }
}

// (G, P) of the supported lengths; false when n has none
bool zmr_split(int n, int *G, int *P);
template <typename T>
void zmr_launch(int n, unsigned grid, int threads, size_t lds, hipStream_t st, cplx<T> *data,
                const cplx<T> *tw, const cplx<T> *khat, const ZRArgs &a);

}  // namespace dda
