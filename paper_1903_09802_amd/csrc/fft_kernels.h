// FFT kernels along the contiguous (x) axis, a strided axis, and the fused z pass of the
// BTTB product.  Included by the translation units that launch them.
#pragma once

#include <algorithm>
#include <type_traits>

#include "fft_engine.h"

namespace dda {

// ---------------------------------------------------------------------------- row (x-axis) FFT

// Field vectors outside the transforms are compact: [R][3][nocc], one entry per occupied
// voxel in voxel order; cidx[voxel] is the entry's index, -1 in air.
enum RowMode {
  ROW_PLAIN = 0,  // in/out: T work rows (setup transforms)
  ROW_OP_FWD,     // in: compact FP64 field (optionally scaled), zero in air and padding; out: T rows
  ROW_OP_INV,     // in: T rows; out (compact): alpha^{-1} x - conv, FP64
  ROW_IMG_INV,    // in: T rows; out (compact): conv, FP64
  ROW_PC_FWD,     // in: compact FP64 field, zero in air; out: T rows (unpadded)
  ROW_PC_INV      // in: T rows; out (compact): scale * v, FP64
};

struct RowArgs {
  FftDesc pl;
  long long rows;      // number of rows transformed
  int tw;              // rows per workgroup (LDS columns)
  int nsh;             // log2(n) when n is a power of two, else -1
  int n_in, n_out;     // valid input length (zero padded to n), output length written
  long long in_stride, out_stride;
  int sign;
  const int *cidx;     // [N] compact index of each voxel, -1 in air
  long long nocc;      // occupied voxels (compact length per component)
  long long vox_rows;  // nz * ny: rows per component block
  long long rhs_rows;  // 3 * nz * ny: rows per right-hand side
  int nx;
  long long N;
  const double2 *ainv; // [R][N]
  const double2 *xin;  // FP64 field rows for ROW_OP_INV
  const double *xscale;// per-RHS input scale xscale[r * kMaxM], or null
  double scale;        // output scale of the transform
  const int *act;      // null, or per-right-hand-side flags: the rows of a right-hand side
                       // whose flag is 0 are neither read nor written (inside a solver cycle,
                       // the right-hand sides that have stopped)
};

constexpr int kRowEpt = 8;  // elements per thread of a row tile: tw n <= 8 (tw tpc) threads

template <typename T, int MODE, typename TI, typename TO, int NF>
__global__ void __launch_bounds__(kFftThreads) k_fft_rows(const TI *in, TO *out,
                                                          const cplx<T> *__restrict__ tw,
                                                          RowArgs a) {
  using V = cplx<T>;
  constexpr bool kCompactIn = MODE == ROW_OP_FWD || MODE == ROW_PC_FWD;
  constexpr bool kCompactOut = MODE == ROW_OP_INV || MODE == ROW_IMG_INV || MODE == ROW_PC_INV;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *s = reinterpret_cast<V *>(smem_raw);
  const int tid = threadIdx.x, nt = blockDim.x;
  const int n = a.pl.n;
  const int ld = a.tw + 1;
  const long long row0 = (long long)blockIdx.x * a.tw;
  // right-hand sides that have stopped: their rows are skipped, the block returns if all are.
  // The flags of the tile's right-hand sides (at most 32, checked at launch) are kept as a bit
  // mask, so that no flag is loaded per element.
  bool some_off = false;
  unsigned onmask = ~0u;
  long long rfirst = 0;
  if (a.act) {
    const long long r0 = row0 / a.rhs_rows, r1 = (min(row0 + a.tw, a.rows) - 1) / a.rhs_rows;
    bool any_on = false;
    rfirst = r0;
    onmask = 0u;
    for (long long r = r0; r <= r1; ++r) {
      if (a.act[r]) {
        any_on = true;
        onmask |= 1u << (r - r0);
      } else {
        some_off = true;
      }
    }
    if (!any_on) return;
  }
  auto rhs_on = [&](long long r) { return !some_off || ((onmask >> (r - rfirst)) & 1u) != 0; };
  auto row_on = [&](long long row) { return !some_off || rhs_on(row / a.rhs_rows); };
  // compact modes: row0 + c = blk vox_rows + vrow with blk = 3 r + component, stepped from the
  // tile's first row in 32-bit arithmetic (rows < 2^31, checked at launch)
  int blk0 = 0, vrow0 = 0;
  if constexpr (kCompactIn || kCompactOut) {
    blk0 = (int)(row0 / a.vox_rows);
    vrow0 = (int)(row0 - (long long)blk0 * a.vox_rows);
  }
  auto split = [&](int c, int &blk, int &vrow) {
    const int vr = (int)a.vox_rows;
    vrow = vrow0 + c;
    blk = blk0;
    while (vrow >= vr) {
      vrow -= vr;
      ++blk;
    }
  };
  const int rows_here = (int)min((long long)a.tw, a.rows - row0);  // rows of this tile
  // load: consecutive threads take consecutive elements of a row (global rows are contiguous)
  const int tot_in = a.tw * n;
  if constexpr (kCompactIn) {
    // compact input: the index-map loads of the thread, then its value loads, then the LDS
    // stores.  Loads are unconditional (from entry 0 where there is nothing to read), air is
    // blended in as a factor 0 and -1 indices are formed by bit operations, so that no load
    // waits behind a branch (at most kRowEpt elements per thread, checked at launch).
    int cis[kRowEpt], bq[kRowEpt];
#pragma unroll
    for (int q = 0; q < kRowEpt; ++q) {
      const int e = tid + q * nt;
      const int c = a.nsh >= 0 ? (e >> a.nsh) : e / n;
      const int i = e - c * n;
      // elements past the tile's last row keep the first row's block, so that the per-block
      // loads below (the input scale) stay inside their arrays
      int blk = blk0, vrow = vrow0;
      if (e < tot_in && c < rows_here) split(c, blk, vrow);
      bq[q] = blk;
      const bool ok = e < tot_in && c < rows_here && i < a.n_in && rhs_on(blk / 3);
      const int ci = a.cidx[ok ? vrow * a.nx + i : 0];
      cis[q] = ci | -(int)!ok;  // -1 where nothing is read
    }
    double2 xv[kRowEpt];
    auto load_values = [&](auto scaled) {
#pragma unroll
      for (int q = 0; q < kRowEpt; ++q) {
        const bool has = cis[q] >= 0;
        xv[q] = in[has ? (long long)bq[q] * a.nocc + cis[q] : 0LL];
        if constexpr (decltype(scaled)::value) xv[q] = cscale(xv[q], a.xscale[(bq[q] / 3) * kMaxM]);
        const double w = has ? 1.0 : 0.0;
        xv[q] = make_double2(xv[q].x * w, xv[q].y * w);
      }
    };
    if (a.xscale) load_values(std::true_type{});
    else load_values(std::false_type{});
#pragma unroll
    for (int q = 0; q < kRowEpt; ++q) {
      const int e = tid + q * nt;
      if (e >= tot_in) continue;
      const int c = a.nsh >= 0 ? (e >> a.nsh) : e / n;
      const int i = e - c * n;
      s[lrow(i, ld) + c] = to_c(xv[q], V{});
    }
  } else {
    // all of the thread's loads, unconditional (from entry 0 past the rows or the input
    // length, blended in as 0), before its LDS stores
    V vals[kRowEpt];
#pragma unroll
    for (int q = 0; q < kRowEpt; ++q) {
      const int e = tid + q * nt;
      const int c = a.nsh >= 0 ? (e >> a.nsh) : e / n;
      const int i = e - c * n;
      const bool ok = e < tot_in && c < rows_here && i < a.n_in;
      const V v = in[ok ? (row0 + c) * a.in_stride + i : 0LL];
      const T w = ok ? (T)1 : (T)0;
      vals[q] = mk<T>(v.x * w, v.y * w);
    }
#pragma unroll
    for (int q = 0; q < kRowEpt; ++q) {
      const int e = tid + q * nt;
      if (e >= tot_in) continue;
      const int c = a.nsh >= 0 ? (e >> a.nsh) : e / n;
      const int i = e - c * n;
      s[lrow(i, ld) + c] = vals[q];
    }
  }
  __syncthreads();
  const Lane L = make_lane(a.tw, tpc_of(n));
  lds_fft_any<V, EptOf<T>::value, NF>(s, ld, L, a.pl, tw, a.sign);
  const int tot_out = a.tw * a.n_out;
  if constexpr (kCompactOut) {
    // compact output: the index-map loads, then the inputs of the update (unconditional, from
    // entry 0 where nothing is written), then the stores of the occupied voxels
    int ciq[kRowEpt], bq[kRowEpt], vq[kRowEpt];
#pragma unroll
    for (int q = 0; q < kRowEpt; ++q) {
      const int e = tid + q * nt;
      const int c = e / a.n_out;
      const int i = e - c * a.n_out;
      int blk = blk0, vrow = vrow0;  // past the last row: the first row's block (see above)
      if (e < tot_out && c < rows_here) split(c, blk, vrow);
      bq[q] = blk;
      vq[q] = vrow * a.nx + i;
      const bool ok = e < tot_out && c < rows_here && rhs_on(blk / 3);
      const int ci = a.cidx[ok ? vq[q] : 0];
      ciq[q] = ci | -(int)!ok;
    }
    double2 xq[kRowEpt], aq[kRowEpt];
    if constexpr (MODE == ROW_OP_INV) {
      auto load_inputs = [&](auto scaled) {
#pragma unroll
        for (int q = 0; q < kRowEpt; ++q) {
          const bool has = ciq[q] >= 0;
          const int r = bq[q] / 3;
          xq[q] = a.xin[has ? (long long)bq[q] * a.nocc + ciq[q] : 0LL];
          if constexpr (decltype(scaled)::value) xq[q] = cscale(xq[q], a.xscale[r * kMaxM]);
          aq[q] = a.ainv[has ? (long long)r * a.N + vq[q] : 0LL];
        }
      };
      if (a.xscale) load_inputs(std::true_type{});
      else load_inputs(std::false_type{});
    }
#pragma unroll
    for (int q = 0; q < kRowEpt; ++q) {
      const int e = tid + q * nt;
      if (e >= tot_out || ciq[q] < 0) continue;
      const int c = e / a.n_out;
      const int i = e - c * a.n_out;
      const double2 conv = cscale(to_d(s[lrow(i, ld) + c]), a.scale);
      double2 y = conv;
      if constexpr (MODE == ROW_OP_INV) y = csub(cmul(aq[q], xq[q]), conv);
      out[(long long)bq[q] * a.nocc + ciq[q]] = y;
    }
  } else {
    for (int e = tid; e < tot_out; e += nt) {
      const int c = e / a.n_out;
      const int i = e - c * a.n_out;
      const long long row = row0 + c;
      if (row >= a.rows || !row_on(row)) continue;
      out[row * a.out_stride + i] = s[lrow(i, ld) + c];
    }
  }
}

// ---------------------------------------------------------------------------- strided-axis FFT

// Data [batch][len][width] (width contiguous); transform along len.  A tile is tw consecutive
// columns of one batch; tiles are numbered batch-major and a workgroup transforms tpw
// consecutive tiles, issuing the next tile's loads before it transforms the current one.
struct StrArgs {
  FftDesc pl;
  long long batch;
  long long width;
  int tw;                 // columns per tile
  long long ntiles;       // ceil(width / tw) tiles per batch
  int tpw;                // tiles per workgroup
  int n_in, n_out;
  long long in_bstride, out_bstride;  // elements between batches
  int sign;
  const int *act;         // null, or per-right-hand-side flags (as RowArgs::act)
  long long rhs_batch;    // batches per right-hand side (with act)
};

template <typename T, int NF>
__global__ void __launch_bounds__(kFftThreads) k_fft_strided(const cplx<T> *in, cplx<T> *out,
                                                             const cplx<T> *__restrict__ tw,
                                                             StrArgs a) {
  using V = cplx<T>;
  constexpr int EPT = EptOf<T>::value;  // rows per thread: n <= EPT tpc
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *s = reinterpret_cast<V *>(smem_raw);
  const int n = a.pl.n;
  const int ld = a.tw + 1;
  const Lane L = make_lane(a.tw, tpc_of(n));
  const long long q0 = (long long)blockIdx.x * a.tpw;
  const long long q1 = min(q0 + a.tpw, a.ntiles * a.batch);
  auto load = [&](long long q, V (&v)[EPT]) {
    const long long b = q / a.ntiles;
    const long long c0 = (q - b * a.ntiles) * (long long)a.tw;
    const bool colok = L.active && (c0 + L.c < a.width);
    const V *src = in + b * a.in_bstride + c0 + L.c;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = L.jt + k * L.tpc;
      v[k] = (colok && i < a.n_in) ? src[(long long)i * a.width] : mk<T>((T)0, (T)0);
    }
  };
  // tiles of right-hand sides that have stopped are skipped (uniformly over the workgroup)
  auto tile_on = [&](long long q) { return !a.act || a.act[(q / a.ntiles) / a.rhs_batch] != 0; };
  V cur[EPT], nxt[EPT];
  if (q0 < q1 && tile_on(q0)) load(q0, cur);
  for (long long q = q0; q < q1; ++q) {
    if (q + 1 < q1 && tile_on(q + 1)) load(q + 1, nxt);  // in flight during this tile's transform
    if (!tile_on(q)) {
#pragma unroll
      for (int k = 0; k < EPT; ++k) cur[k] = nxt[k];
      continue;
    }
    if (q > q0) lds_barrier();         // the previous tile's output reads are done
    if (L.active) {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int i = L.jt + k * L.tpc;
        if (i < n) s[lrow(i, ld) + L.c] = cur[k];
      }
    }
    lds_barrier();
    lds_fft_any<V, EPT, NF>(s, ld, L, a.pl, tw, a.sign);
    const long long b = q / a.ntiles;
    const long long c0 = (q - b * a.ntiles) * (long long)a.tw;
    V *dst = out + b * a.out_bstride + c0 + L.c;
    if (L.active && c0 + L.c < a.width)
      for (int i = L.jt; i < a.n_out; i += L.tpc) dst[(long long)i * a.width] = s[lrow(i, ld) + L.c];
#pragma unroll
    for (int k = 0; k < EPT; ++k) cur[k] = nxt[k];
  }
}

// ---------------------------------------------------------------------------- fused z pass

// Data [R][3][nz][zstride]: z rows of plane = 2ny * 2nx columns (after the x and y
// transforms), zstride >= plane.  For a
// tile of `tw` consecutive (ky, kx) columns of one right-hand side: zero-pad each of
// the three components to 2nz along z, FFT, multiply by the 3x3 symmetric kernel
// spectrum (six components, read from the stored octant with the per-axis parity
// signs), inverse FFT, write the first nz entries back in place.  tw is a power of two.
struct ZArgs {
  FftDesc pl;       // length 2nz
  int nz, ny, nx;
  long long plane;  // 4 nx ny columns
  long long zstride;  // elements between z rows (>= plane)
  int tw, twsh;     // columns per tile and log2(tw)
  long long ntiles;
  long long nrhs;
  const int *act;   // null, or per-right-hand-side flags (as RowArgs::act)
};

template <typename T, int EPT, int NF>
__global__ void __launch_bounds__(768) k_zpass(cplx<T> *data, const cplx<T> *__restrict__ tw,
                                               const cplx<T> *__restrict__ khat, ZArgs a) {
  using V = cplx<T>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  V *s = reinterpret_cast<V *>(smem_raw);
  const int n = a.pl.n;
  const int ncols = 3 * a.tw;
  const int ld = ncols + 1;
  const long long blk = xcd_remap(blockIdx.x, a.ntiles * a.nrhs);
  if (blk >= a.ntiles * a.nrhs) return;
  // right-hand sides fastest: the workgroups that read the same kernel-spectrum columns are
  // adjacent and, through the XCD remap, share one L2
  const long long r = blk % a.nrhs;
  if (a.act && !a.act[r]) return;
  const long long c0 = (blk / a.nrhs) * (long long)a.tw;
  V *base = data + r * 3LL * a.nz * a.zstride;
  const Lane L = make_lane(ncols, tpc_of(n));
  if (L.active) {
    const int comp = L.c >> a.twsh, c = L.c & (a.tw - 1);
    const bool ok = c0 + c < a.plane;
    const V *src = base + (long long)comp * a.nz * a.zstride + c0 + c;
    for (int i = L.jt; i < n; i += L.tpc) {
      V val = mk<T>((T)0, (T)0);
      if (i < a.nz && ok) val = src[(long long)i * a.zstride];
      s[lrow(i, ld) + L.c] = val;
    }
  }
  __syncthreads();
  lds_fft_any<V, EPT, NF>(s, ld, L, a.pl, tw, -1);
  // pointwise 3x3 multiply: thread -> column tid % tw, rows tid / tw + q (blockDim / tw)
  {
    const int L2x = 2 * a.nx;
    const long long ox_n = a.nx + 1, oy_n = a.ny + 1;
    const long long cstride = (long long)(a.nz + 1) * oy_n * ox_n;
    const int c = threadIdx.x & (a.tw - 1);
    const int rstep = blockDim.x >> a.twsh;
    const long long kyx = c0 + c;
    if (kyx < a.plane) {
      const int ky = (int)(kyx / L2x);
      const int kx = (int)(kyx - (long long)ky * L2x);
      int mxy = 0;
      int ox = kx, oy = ky;
      if (kx > a.nx) { ox = L2x - kx; mxy |= 1; }
      if (ky > a.ny) { oy = 2 * a.ny - ky; mxy |= 2; }
      for (int i = threadIdx.x >> a.twsh; i < n; i += rstep) {
        int mir = mxy, oz = i;
        if (i > a.nz) { oz = n - i; mir |= 4; }
        const long long o = ((long long)oz * oy_n + oy) * ox_n + ox;
        V K[6];
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) {
          V kv = khat[cc * cstride + o];
          if (__popc(comp_odd_mask(cc) & mir) & 1) { kv.x = -kv.x; kv.y = -kv.y; }
          K[cc] = kv;
        }
        V *row = s + lrow(i, ld);
        const V x0 = row[c], x1 = row[a.tw + c], x2 = row[2 * a.tw + c];
        row[c] = cadd(cadd(cmul(K[0], x0), cmul(K[1], x1)), cmul(K[2], x2));
        row[a.tw + c] = cadd(cadd(cmul(K[1], x0), cmul(K[3], x1)), cmul(K[4], x2));
        row[2 * a.tw + c] = cadd(cadd(cmul(K[2], x0), cmul(K[4], x1)), cmul(K[5], x2));
      }
    }
  }
  __syncthreads();
  lds_fft_any<V, EPT, NF>(s, ld, L, a.pl, tw, +1);
  if (L.active) {
    const int comp = L.c >> a.twsh, c = L.c & (a.tw - 1);
    if (c0 + c < a.plane) {
      V *dst = base + (long long)comp * a.nz * a.zstride + c0 + c;
      for (int i = L.jt; i < a.nz; i += L.tpc) dst[(long long)i * a.zstride] = s[lrow(i, ld) + L.c];
    }
  }
}

// ---------------------------------------------------------------------------- host helpers

inline void set_lds_limit(const void *fn, size_t bytes) {
  if (bytes > 48 * 1024) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename T> inline const cplx<T> *tw_of(const FftPlan &p);
template <> inline const double2 *tw_of<double>(const FftPlan &p) { return p.tw64; }
template <> inline const float2 *tw_of<float>(const FftPlan &p) { return p.tw32; }

// Call f(std::integral_constant<int, NF>) with NF = n for the lengths that have a
// compile-time plan (powers of two 16 .. 512 and the mixed lengths 80, 96, 112, 160, 192),
// NF = 0 (runtime plan) otherwise.
template <typename F> inline void with_static_n(int n, F &&f) {
  switch (n) {
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    case 128: f(std::integral_constant<int, 128>{}); break;
    case 256: f(std::integral_constant<int, 256>{}); break;
    case 512: f(std::integral_constant<int, 512>{}); break;
    case 80: f(std::integral_constant<int, 80>{}); break;
    case 96: f(std::integral_constant<int, 96>{}); break;
    case 112: f(std::integral_constant<int, 112>{}); break;
    case 160: f(std::integral_constant<int, 160>{}); break;
    case 192: f(std::integral_constant<int, 192>{}); break;
    default: f(std::integral_constant<int, 0>{}); break;
  }
}

inline int ilog2_exact(int n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int s = 0;
  while ((1 << s) < n) ++s;
  return s;
}

// Columns per tile for a length-n transform: fill 256 threads (tpc threads per column)
// within a 40 KB LDS tile.
template <typename T> inline int tile_cols(int n) {
  const int tpc = tpc_of(n);
  int t = kFftThreads / tpc;
  if (t < 1) t = 1;
  while (t > 1 && (size_t)lds_elems(n, t + 1) * sizeof(cplx<T>) > 40 * 1024) --t;
  return t;
}

template <typename T> inline size_t tile_lds(int n, int cols) {
  return (size_t)lds_elems(n, cols + 1) * sizeof(cplx<T>);
}

// Launch a row transform.  `a` must have rows, n_in, n_out, strides and sign set.
// `pass` (an FftPass, or -1) selects the autotuned rows per tile.
template <typename T, int MODE, typename TI, typename TO>
inline void launch_rows(dda_problem *p, const FftPlan &pl, const TI *in, TO *out, RowArgs a,
                        const char *name, double bytes, int pass = -1) {
  a.pl = desc(pl);
  a.act = a.rhs_rows > 0 ? p->act : nullptr;
  a.tw = tile_cols<T>(pl.n);
  if (pass >= 0) {
    const TileShape &ts = p->tile[pass][sizeof(T) == 8 ? 0 : 1];
    if (ts.tw > 0 && ts.tw < a.tw) a.tw = ts.tw;
  }
  if (a.rows < a.tw) a.tw = (int)a.rows;
  // a tile spans at most 32 right-hand sides (the kernel keeps their flags as a bit mask)
  if (a.rhs_rows > 0 && a.tw > 30 * a.rhs_rows) a.tw = (int)(30 * a.rhs_rows);
  a.nsh = ilog2_exact(pl.n);
  const long long blocks = (a.rows + a.tw - 1) / a.tw;
  const size_t lds = tile_lds<T>(pl.n, a.tw);
  const int threads = std::max(64, a.tw * tpc_of(pl.n));
  REQUIRE((long long)a.tw * pl.n <= (long long)kRowEpt * threads, DDA_EUNSUPPORTED,
          "row tile of %d x %d exceeds %d elements per thread", a.tw, pl.n, kRowEpt);
  REQUIRE(a.rows < (1LL << 31) && (a.rhs_rows == 0 || a.rhs_rows == 3 * a.vox_rows), DDA_EUNSUPPORTED,
          "row transform of %lld rows", a.rows);
  KTimer t(&p->prof, p->st, name, bytes);
  with_static_n(pl.n, [&](auto nf) {
    auto fn = k_fft_rows<T, MODE, TI, TO, decltype(nf)::value>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)blocks), dim3(threads), lds, p->st, in, out,
                       tw_of<T>(pl), a);
  });
  HIPCHK(hipGetLastError());
}

// `pass` (an FftPass, or -1) selects the autotuned columns per tile and tiles per workgroup.
template <typename T>
inline void launch_strided(dda_problem *p, const FftPlan &pl, const cplx<T> *in, cplx<T> *out,
                           long long batch, long long width, int n_in, int n_out,
                           long long in_bstride, long long out_bstride, int sign,
                           const char *name, double bytes, long long rhs_batch = 0, int pass = -1) {
  StrArgs a;
  a.pl = desc(pl);
  a.batch = batch;
  a.width = width;
  a.tw = tile_cols<T>(pl.n);
  TileShape ts;
  if (pass >= 0) ts = p->tile[pass][sizeof(T) == 8 ? 0 : 1];
  if (ts.tw > 0 && ts.tw < a.tw) a.tw = ts.tw;
  if (a.tw > width) a.tw = (int)width;
  a.ntiles = (width + a.tw - 1) / a.tw;
  // tiles per workgroup: the most (up to 8) that leave at least 2048 workgroups, or the tuned count
  const long long tiles = a.ntiles * batch;
  a.tpw = 1;
  while (a.tpw < 8 && (tiles + 2 * a.tpw - 1) / (2 * a.tpw) >= 2048) a.tpw *= 2;
  if (ts.tpw > 0) a.tpw = ts.tpw;
  a.n_in = n_in;
  a.n_out = n_out;
  a.in_bstride = in_bstride;
  a.out_bstride = out_bstride;
  a.sign = sign;
  a.act = rhs_batch > 0 ? p->act : nullptr;
  a.rhs_batch = rhs_batch > 0 ? rhs_batch : 1;
  const size_t lds = tile_lds<T>(pl.n, a.tw);
  const int threads = a.tw * tpc_of(pl.n);
  KTimer t(&p->prof, p->st, name, bytes);
  with_static_n(pl.n, [&](auto nf) {
    auto fn = k_fft_strided<T, decltype(nf)::value>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)((tiles + a.tpw - 1) / a.tpw)), dim3(threads), lds, p->st,
                       in, out, tw_of<T>(pl), a);
  });
  HIPCHK(hipGetLastError());
}

}  // namespace dda
