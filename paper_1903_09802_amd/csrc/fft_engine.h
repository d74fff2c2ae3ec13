// LDS-resident mixed-radix FFT engine for CDNA (wave64) workgroups.
//
// A workgroup holds `ncols` independent sequences of length n in LDS, element
// (i, c) at s[i * ld + c] (ld >= ncols).  Each radix pass is a Stockham
// autosort step: butterfly j of a pass with radix R and accumulated span Ns
// reads x[j + r n/R], twiddles by exp(sign 2 pi i r (j mod Ns) / (Ns R)),
// applies the R-point DFT and writes x[(j / Ns) Ns R + (j mod Ns) + r Ns]; the
// output is in natural order.  All reads of a pass finish (barrier) before any
// write, so one LDS buffer suffices.  Threads are mapped column-fastest, so a
// wave touches contiguous 128-byte LDS rows (no bank conflicts for complex
// double / float).  Each thread holds at most EPT complex values per pass.
#pragma once

#include "common.h"

namespace dda {

template <typename V> struct RealOf;
template <> struct RealOf<double2> { using type = double; };
template <> struct RealOf<float2> { using type = float; };

// R-point DFT in registers; sign = -1 forward, +1 inverse (unnormalised).
template <int R, typename V>
__device__ __forceinline__ void dft(V *a, int sign) {
  using T = typename RealOf<V>::type;
  if constexpr (R == 2) {
    V t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  } else if constexpr (R == 3) {
    const T c3 = (T)0.8660254037844386;
    V t1 = cadd(a[1], a[2]);
    V t2 = csub(a[1], a[2]);
    V m = csub(a[0], cscale(t1, (T)0.5));
    V q = cmuli(cscale(t2, c3), sign);
    a[0] = cadd(a[0], t1);
    a[1] = cadd(m, q);
    a[2] = csub(m, q);
  } else if constexpr (R == 4) {
    V t0 = cadd(a[0], a[2]);
    V t1 = csub(a[0], a[2]);
    V t2 = cadd(a[1], a[3]);
    V t3 = cmuli(csub(a[1], a[3]), sign);
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  } else if constexpr (R == 8) {
    const T h = (T)0.7071067811865475;
    V e[4] = {a[0], a[2], a[4], a[6]};
    V o[4] = {a[1], a[3], a[5], a[7]};
    dft<4, V>(e, sign);
    dft<4, V>(o, sign);
    V o1 = cscale(cadd(o[1], cmuli(o[1], sign)), h);
    V o2 = cmuli(o[2], sign);
    V o3 = cscale(csub(cmuli(o[3], sign), o[3]), h);
    a[0] = cadd(e[0], o[0]);
    a[4] = csub(e[0], o[0]);
    a[1] = cadd(e[1], o1);
    a[5] = csub(e[1], o1);
    a[2] = cadd(e[2], o2);
    a[6] = csub(e[2], o2);
    a[3] = cadd(e[3], o3);
    a[7] = csub(e[3], o3);
  } else if constexpr (R == 5) {
    const T c1 = (T)0.30901699437494745, c2 = (T)-0.8090169943749473;
    const T s1 = (T)0.9510565162951535, s2 = (T)0.5877852522924732;
    V t1 = cadd(a[1], a[4]), d1 = csub(a[1], a[4]);
    V t2 = cadd(a[2], a[3]), d2 = csub(a[2], a[3]);
    V r1 = cadd(a[0], cadd(cscale(t1, c1), cscale(t2, c2)));
    V r2 = cadd(a[0], cadd(cscale(t1, c2), cscale(t2, c1)));
    V i1 = cmuli(cadd(cscale(d1, s1), cscale(d2, s2)), sign);
    V i2 = cmuli(csub(cscale(d1, s2), cscale(d2, s1)), sign);
    a[0] = cadd(a[0], cadd(t1, t2));
    a[1] = cadd(r1, i1);
    a[4] = csub(r1, i1);
    a[2] = cadd(r2, i2);
    a[3] = csub(r2, i2);
  } else if constexpr (R == 7) {
    // cos / sin of 2 pi m / 7, m = 0..6
    const T C[7] = {(T)1.0, (T)0.6234898018587336, (T)-0.22252093395631434, (T)-0.900968867902419,
                    (T)-0.900968867902419, (T)-0.22252093395631434, (T)0.6234898018587336};
    const T S[7] = {(T)0.0, (T)0.7818314824680298, (T)0.9749279121818236, (T)0.43388373911755823,
                    (T)-0.43388373911755823, (T)-0.9749279121818236, (T)-0.7818314824680298};
    V t[4], dd[4];
#pragma unroll
    for (int q = 1; q <= 3; ++q) {
      t[q] = cadd(a[q], a[7 - q]);
      dd[q] = csub(a[q], a[7 - q]);
    }
    V out[7];
    out[0] = cadd(a[0], cadd(t[1], cadd(t[2], t[3])));
#pragma unroll
    for (int kk = 1; kk <= 3; ++kk) {
      V re = a[0];
      V im = mk<T>((T)0, (T)0);
#pragma unroll
      for (int q = 1; q <= 3; ++q) {
        const int mm = (q * kk) % 7;
        re = cadd(re, cscale(t[q], C[mm]));
        im = cadd(im, cscale(dd[q], S[mm]));
      }
      V iv = cmuli(im, sign);
      out[kk] = cadd(re, iv);
      out[7 - kk] = csub(re, iv);
    }
#pragma unroll
    for (int q = 0; q < 7; ++q) a[q] = out[q];
  }
}

// One Stockham pass of radix R over all columns.
template <int R, typename V, int EPT>
__device__ __forceinline__ void fft_pass(V *s, int ld, int ncols, int n, int Ns,
                                         const V *__restrict__ tw, int sign, int tid,
                                         int nthreads) {
  constexpr int BPT = (EPT + R - 1) / R;
  V v[BPT][R];
  const int nb = n / R;
  const int total = nb * ncols;
  const int twstep = n / (Ns * R);
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * nthreads;
    if (b < total) {
      const int c = b % ncols;
      const int j = b / ncols;
      const int kk = j % Ns;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = s[(j + r * nb) * ld + c];
      if (kk != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w = tw[r * kk * twstep];
          if (sign > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      dft<R, V>(v[q], sign);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int b = tid + q * nthreads;
    if (b < total) {
      const int c = b % ncols;
      const int j = b / ncols;
      const int kk = j % Ns;
      const int base = (j / Ns) * Ns * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) s[(base + r * Ns) * ld + c] = v[q][r];
    }
  }
  __syncthreads();
}

// Full transform of ncols columns (caller synchronises before the call).
template <typename V, int EPT>
__device__ __forceinline__ void lds_fft(V *s, int ld, int ncols, const FftDesc &pl,
                                        const V *__restrict__ tw, int sign, int tid,
                                        int nthreads) {
  int Ns = 1;
  for (int ps = 0; ps < pl.nrad; ++ps) {
    const int R = pl.rad[ps];
    switch (R) {
      case 2: fft_pass<2, V, EPT>(s, ld, ncols, pl.n, Ns, tw, sign, tid, nthreads); break;
      case 3: fft_pass<3, V, EPT>(s, ld, ncols, pl.n, Ns, tw, sign, tid, nthreads); break;
      case 4: fft_pass<4, V, EPT>(s, ld, ncols, pl.n, Ns, tw, sign, tid, nthreads); break;
      case 5: fft_pass<5, V, EPT>(s, ld, ncols, pl.n, Ns, tw, sign, tid, nthreads); break;
      case 7: fft_pass<7, V, EPT>(s, ld, ncols, pl.n, Ns, tw, sign, tid, nthreads); break;
      default: fft_pass<8, V, EPT>(s, ld, ncols, pl.n, Ns, tw, sign, tid, nthreads); break;
    }
    Ns *= R;
  }
}

// Elements per thread per pass: 8 complex doubles or 16 complex floats (32 KB tiles at 256 threads).
template <typename T> struct EptOf;
template <> struct EptOf<double> { static constexpr int value = 8; };
template <> struct EptOf<float> { static constexpr int value = 16; };

constexpr int kFftThreads = 256;

}  // namespace dda
