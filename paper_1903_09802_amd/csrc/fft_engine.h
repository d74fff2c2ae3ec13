// LDS-resident mixed-radix FFT engine for CDNA (wave64) workgroups.
//
// A workgroup holds `ncols` independent sequences of length n in LDS; element (i, c) sits at
// s[lrow(i, ld) + c] with lrow(i) = i * ld + (i >> 3): rows are padded to ld >= ncols + 1 and
// every eighth row is skewed by one more element, so the stride-R row accesses of a radix-R
// pass spread over the LDS banks.  Each radix pass is a Stockham autosort step: butterfly j
// of a pass with radix R and accumulated span Ns reads x[j + r n/R], twiddles by
// exp(sign 2 pi i r (j mod Ns) / (Ns R)), applies the R-point DFT and writes
// x[(j / Ns) Ns R + (j mod Ns) + r Ns]; the output is in natural order.  All reads of a
// pass finish (barrier) before any write, so one LDS buffer suffices.
//
// Thread mapping: thread t owns column c = t % ncols and row slot jt = t / ncols (computed
// once); with TPC threads per column it handles butterflies j = jt + q TPC.  When Ns is a
// power of two the span arithmetic is shifts and masks.
#pragma once

#include "common.h"

namespace dda {

// Workgroup barrier for LDS traffic only: it orders the workgroup's LDS accesses without
// waiting for its outstanding global loads, so a prefetch stays in flight across it.  Every
// global value these kernels load is consumed (written to LDS or used) before the barrier
// that publishes it, so cross-thread reuse of global addresses stays ordered.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename V> struct RealOf;
template <> struct RealOf<double2> { using type = double; };
template <> struct RealOf<float2> { using type = float; };

__host__ __device__ __forceinline__ int lrow(int i, int ld) { return i * ld + (i >> 3); }
// LDS elements for n rows of stride ld
__host__ __device__ __forceinline__ int lds_elems(int n, int ld) { return lrow(n, ld) + 1; }

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

// Per-thread placement inside a tile: column c, first butterfly row jt, TPC threads per column.
struct Lane {
  int c, jt, tpc, active;
};

__device__ __forceinline__ Lane make_lane(int ncols, int tpc) {
  Lane L;
  L.c = threadIdx.x % ncols;
  L.jt = threadIdx.x / ncols;
  L.tpc = tpc;
  L.active = L.jt < tpc;
  return L;
}

// One Stockham pass of radix R over all columns.
template <int R, typename V, int EPT>
__device__ __forceinline__ void fft_pass(V *s, int ld, const Lane &L, int n, int Ns, int nsh,
                                         const V *__restrict__ tw, int sign) {
  constexpr int BPT = (EPT + R - 1) / R;
  V v[BPT][R];
  const int nb = n / R;
  const int twstep = n / (Ns * R);
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int j = L.jt + q * L.tpc;
    if (L.active && j < nb) {
      const int kk = nsh >= 0 ? (j & (Ns - 1)) : (j % Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = s[lrow(j + r * nb, ld) + L.c];
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
  lds_barrier();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int j = L.jt + q * L.tpc;
    if (L.active && j < nb) {
      int base;
      if (nsh >= 0) base = ((j >> nsh) << nsh) * R + (j & (Ns - 1));
      else base = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
      for (int r = 0; r < R; ++r) s[lrow(base + r * Ns, ld) + L.c] = v[q][r];
    }
  }
  lds_barrier();
}

// Full transform of all columns (caller synchronises before the call).
template <typename V, int EPT>
__device__ __forceinline__ void lds_fft(V *s, int ld, const Lane &L, const FftDesc &pl,
                                        const V *__restrict__ tw, int sign) {
  int Ns = 1, nsh = 0;
  for (int ps = 0; ps < pl.nrad; ++ps) {
    const int R = pl.rad[ps];
    switch (R) {
      case 2: fft_pass<2, V, EPT>(s, ld, L, pl.n, Ns, nsh, tw, sign); break;
      case 3: fft_pass<3, V, EPT>(s, ld, L, pl.n, Ns, nsh, tw, sign); break;
      case 4: fft_pass<4, V, EPT>(s, ld, L, pl.n, Ns, nsh, tw, sign); break;
      case 5: fft_pass<5, V, EPT>(s, ld, L, pl.n, Ns, nsh, tw, sign); break;
      case 7: fft_pass<7, V, EPT>(s, ld, L, pl.n, Ns, nsh, tw, sign); break;
      default: fft_pass<8, V, EPT>(s, ld, L, pl.n, Ns, nsh, tw, sign); break;
    }
    Ns *= R;
    if (nsh >= 0) nsh = (R == 2) ? nsh + 1 : (R == 4) ? nsh + 2 : (R == 8) ? nsh + 3 : -1;
  }
}

// Elements per thread per pass: 8 complex values (one radix-8 butterfly).
constexpr int kEpt = 8;
template <typename T> struct EptOf { static constexpr int value = kEpt; };

// Threads per column for a length-n transform.
__host__ __device__ __forceinline__ int tpc_of(int n) { return (n + kEpt - 1) / kEpt; }

// ---------------------------------------------------------------------------- static plans
// 7-smooth lengths with the radix plan fixed at compile time (8s, then a 4 or a 2, then 3s,
// 5s and 7s): the spans, strides and twiddle steps become constants.

__host__ __device__ constexpr int st_nrad(int n) {
  int k = 0, m = n;
  while (m % 8 == 0) { m /= 8; ++k; }
  if (m % 4 == 0) { m /= 4; ++k; }
  if (m % 2 == 0) { m /= 2; ++k; }
  while (m % 3 == 0) { m /= 3; ++k; }
  while (m % 5 == 0) { m /= 5; ++k; }
  while (m % 7 == 0) { m /= 7; ++k; }
  return k;
}
__host__ __device__ constexpr int st_rad(int n, int p) {
  int m = n, k = 0;
  while (m % 8 == 0) { if (k == p) return 8; m /= 8; ++k; }
  if (m % 4 == 0) { if (k == p) return 4; m /= 4; ++k; }
  if (m % 2 == 0) { if (k == p) return 2; m /= 2; ++k; }
  while (m % 3 == 0) { if (k == p) return 3; m /= 3; ++k; }
  while (m % 5 == 0) { if (k == p) return 5; m /= 5; ++k; }
  while (m % 7 == 0) { if (k == p) return 7; m /= 7; ++k; }
  return 1;
}
static_assert(st_nrad(192) == 3 && st_rad(192, 0) == 8 && st_rad(192, 1) == 8 && st_rad(192, 2) == 3);
static_assert(st_nrad(80) == 3 && st_rad(80, 1) == 2 && st_rad(80, 2) == 5);
static_assert(st_nrad(112) == 3 && st_rad(112, 2) == 7 && st_nrad(256) == 3 && st_rad(256, 2) == 4);

template <int R, typename V, int N, int NS>
__device__ __forceinline__ void fft_pass_s(V *s, int ld, const Lane &L, const V *__restrict__ tw,
                                           int sign) {
  constexpr int BPT = (kEpt + R - 1) / R;
  constexpr int NB = N / R;
  constexpr int TPC = (N + kEpt - 1) / kEpt;
  constexpr int TWSTEP = N / (NS * R);
  V v[BPT][R];
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int j = L.jt + q * TPC;
    if (L.active && j < NB) {
      const int kk = j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = s[lrow(j + r * NB, ld) + L.c];
      if (NS > 1 && kk != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          V w = tw[r * kk * TWSTEP];
          if (sign > 0) w.y = -w.y;
          v[q][r] = cmul(v[q][r], w);
        }
      }
      dft<R, V>(v[q], sign);
    }
  }
  lds_barrier();
#pragma unroll
  for (int q = 0; q < BPT; ++q) {
    const int j = L.jt + q * TPC;
    if (L.active && j < NB) {
      const int base = (j / NS) * (NS * R) + j % NS;
#pragma unroll
      for (int r = 0; r < R; ++r) s[lrow(base + r * NS, ld) + L.c] = v[q][r];
    }
  }
  lds_barrier();
}

template <typename V, int N, int P = 0, int NS = 1>
__device__ __forceinline__ void lds_fft_s(V *s, int ld, const Lane &L, const V *__restrict__ tw,
                                          int sign) {
  if constexpr (P < st_nrad(N)) {
    constexpr int R = st_rad(N, P);
    fft_pass_s<R, V, N, NS>(s, ld, L, tw, sign);
    lds_fft_s<V, N, P + 1, NS * R>(s, ld, L, tw, sign);
  }
}

// Transform with the static plan when NF > 0 (NF must equal pl.n), else the runtime plan.
template <typename V, int EPT, int NF>
__device__ __forceinline__ void lds_fft_any(V *s, int ld, const Lane &L, const FftDesc &pl,
                                            const V *__restrict__ tw, int sign) {
  if constexpr (NF > 0) lds_fft_s<V, NF>(s, ld, L, tw, sign);
  else lds_fft<V, EPT>(s, ld, L, pl, tw, sign);
}

constexpr int kFftThreads = 256;

}  // namespace dda
