// The DDA operator: problem setup (polarisability, incident field), the Green-tensor
// kernel spectrum, and the five-pass zero-padded FFT product (Sec. 1, 2.1-2.2).
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "fft_kernels.h"
#include "zpass_mr.h"

namespace dda {

// d^3 G_ab at displacement (x, y, z), six components xx xy xz yy yz zz (Sec. 2:
// G = e^{ikr}/r [k^2 (I - rr^T) + (ikr - 1)/r^2 (I - 3 rr^T)]).
__device__ __forceinline__ void green6_d3(double x, double y, double z, double k, double d3,
                                          double2 g[6]) {
  const double r2 = x * x + y * y + z * z;
  const double r = sqrt(r2);
  const double ir = 1.0 / r;
  const double h[3] = {x * ir, y * ir, z * ir};
  double sn, cs;
  sincos(k * r, &sn, &cs);
  const double2 e = make_double2(cs * ir * d3, sn * ir * d3);
  const double k2 = k * k;
  const double ir2 = ir * ir;
  const double kr = k * r;
  int c = 0;
  for (int a = 0; a < 3; ++a)
    for (int b = a; b < 3; ++b) {
      const double P = h[a] * h[b];
      const double dl = (a == b) ? 1.0 : 0.0;
      const double re = k2 * (dl - P) - (dl - 3.0 * P) * ir2;
      const double im = kr * (dl - 3.0 * P) * ir2;
      g[c++] = cmul(e, make_double2(re, im));
    }
}

// Embedding of K(p, q, s) = d^3 G(p d, q d, s d) on the (2nx, 2ny, 2nz) circulant grid:
// index i <-> offset i (i < n), i - 2n (i > n); index n (offset +-n, never used) and the
// origin hold 0.
__global__ void k_green_pad(double2 *out, int nx, int ny, int nz, double k, double d) {
  const long long Lx = 2LL * nx, Ly = 2LL * ny, Lz = 2LL * nz;
  const long long tot = Lx * Ly * Lz;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const int ix = (int)(idx % Lx);
  const int iy = (int)((idx / Lx) % Ly);
  const int iz = (int)(idx / (Lx * Ly));
  double2 g[6];
  bool zero = (ix == nx) || (iy == ny) || (iz == nz) || (ix == 0 && iy == 0 && iz == 0);
  if (!zero) {
    const int p = ix < nx ? ix : ix - 2 * nx;
    const int q = iy < ny ? iy : iy - 2 * ny;
    const int s = iz < nz ? iz : iz - 2 * nz;
    green6_d3(p * d, q * d, s * d, k, d * d * d, g);
  } else {
    for (int c = 0; c < 6; ++c) g[c] = make_double2(0.0, 0.0);
  }
  for (int c = 0; c < 6; ++c) out[c * tot + idx] = g[c];
}

// One octant (non-negative offsets) of the padded spectrum: component-major
// [6][nz+1][ny+1][nx+1], or z-major [ny+1][nx+1][nz+1][6] for the register z pass.  IMAG keeps
// the imaginary part as a real spectrum: the embedded kernel is even under r -> -r (every
// component), so its transform is a sum of K against real cosine products, and the imaginary
// part of the spectrum is exactly the spectrum of d^3 Im G.
template <typename TO, bool ZMAJOR, bool IMAG = false>
__global__ void k_extract_octant(const double2 *full, TO *oct, int nx, int ny, int nz) {
  const long long ox_n = nx + 1, oy_n = ny + 1, oz_n = nz + 1;
  const long long per = ox_n * oy_n * oz_n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 6 * per) return;
  int c, ox, oy, oz;
  if (ZMAJOR) {
    c = (int)(idx % 6);
    const long long rem = idx / 6;
    oz = (int)(rem % oz_n);
    ox = (int)((rem / oz_n) % ox_n);
    oy = (int)(rem / (oz_n * ox_n));
  } else {
    c = (int)(idx / per);
    const long long rem = idx - c * per;
    ox = (int)(rem % ox_n);
    oy = (int)((rem / ox_n) % oy_n);
    oz = (int)(rem / (ox_n * oy_n));
  }
  const long long Lx = 2LL * nx, Ly = 2LL * ny, Lz = 2LL * nz;
  double2 v = full[c * Lx * Ly * Lz + ((long long)oz * Ly + oy) * Lx + ox];
  if (IMAG) v = make_double2(v.y, 0.0);
  oct[idx] = to_c(v, TO{});
}

static inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

template <typename TO, bool IMAG = false>
static void extract_octant(dda_problem *p, const double2 *full, TO *oct) {
  const long long n = 6LL * (p->nx + 1) * (p->ny + 1) * (p->nz + 1);
  if (p->zreg)
    hipLaunchKernelGGL((k_extract_octant<TO, true, IMAG>), dim3(nblk(n, 256)), dim3(256), 0, p->st,
                       full, oct, p->nx, p->ny, p->nz);
  else
    hipLaunchKernelGGL((k_extract_octant<TO, false, IMAG>), dim3(nblk(n, 256)), dim3(256), 0, p->st,
                       full, oct, p->nx, p->ny, p->nz);
  HIPCHK(hipGetLastError());
}

// Occupancy, invalid permittivities and the occupied-permittivity sum, per block.
__global__ void k_validate(const uint8_t *mask, const double2 *eps, long long N, double *partial) {
  __shared__ double sh[6][256];
  double occ = 0, bad = 0, sr = 0, si = 0, qr = 0, qi = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    if (mask[i]) {
      const double2 e = eps[i];
      occ += 1.0;
      sr += e.x;
      si += e.y;
      const double d1 = fabs(e.x - 1.0) + fabs(e.y), d2 = fabs(e.x + 2.0) + fabs(e.y);
      if (d1 < 1e-12 || d2 < 1e-12 || !isfinite(e.x) || !isfinite(e.y)) {
        bad += 1.0;
      } else {  // (eps + 2) / (eps - 1), the part of 1/alpha that is not linear in eps
        const double2 q = cdiv(make_double2(e.x + 2.0, e.y), make_double2(e.x - 1.0, e.y));
        qr += q.x;
        qi += q.y;
      }
    }
  }
  sh[0][threadIdx.x] = occ;
  sh[1][threadIdx.x] = bad;
  sh[2][threadIdx.x] = sr;
  sh[3][threadIdx.x] = si;
  sh[4][threadIdx.x] = qr;
  sh[5][threadIdx.x] = qi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 6; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 6; ++q) partial[blockIdx.x * 6 + q] = sh[q][0];
}

__global__ void k_alpha(const uint8_t *mask, const double2 *eps, long long N, double kd,
                        const double *S, double2 *ainv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (i >= N) return;
  ainv[r * N + i] = mask[i] ? ldr_alpha_inv(eps[i], kd, S[r]) : make_double2(0.0, 0.0);
}

// b[r][a][c] = pol_a exp(+-i k dir . r_v) for occupied voxel v = vox[c] (compact layout).
__global__ void k_incident(const int *vox, long long nocc, int nx, int ny, int nz, double k,
                           double d, const double *dirpol, int conj, double2 *b) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= nocc) return;
  const long long i = vox[c];
  const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((long long)nx * ny));
  const double x = (ix - 0.5 * (nx - 1)) * d, y = (iy - 0.5 * (ny - 1)) * d,
               z = (iz - 0.5 * (nz - 1)) * d;
  const double *dp = dirpol + 6 * r;
  const double ph = k * (dp[0] * x + dp[1] * y + dp[2] * z);
  double sn, cs;
  sincos(ph, &sn, &cs);
  if (conj) sn = -sn;
  double2 *br = b + (long long)r * 3 * nocc;
  for (int a = 0; a < 3; ++a) br[a * nocc + c] = make_double2(dp[3 + a] * cs, dp[3 + a] * sn);
}

// Compact index map, pass 1: occupied voxels per block of kMapBlock voxels.
constexpr int kMapBlock = 256;
__global__ void k_map_count(const uint8_t *mask, long long N, int *count) {
  __shared__ int sh[kMapBlock];
  const long long v = (long long)blockIdx.x * kMapBlock + threadIdx.x;
  sh[threadIdx.x] = (v < N && mask[v]) ? 1 : 0;
  __syncthreads();
  for (int s = kMapBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[blockIdx.x] = sh[0];
}

// Pass 2: with the exclusive prefix of the block counts, cidx[v] = compact index (or -1) and
// vox[c] = voxel of compact entry c (a block-local inclusive scan gives the ranks).
__global__ void k_map_fill(const uint8_t *mask, long long N, const long long *base, int *cidx,
                           int *vox) {
  __shared__ int sh[kMapBlock];
  const long long v = (long long)blockIdx.x * kMapBlock + threadIdx.x;
  const int occ = (v < N && mask[v]) ? 1 : 0;
  sh[threadIdx.x] = occ;
  __syncthreads();
  for (int off = 1; off < kMapBlock; off <<= 1) {  // Hillis-Steele inclusive scan
    const int t = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (v >= N) return;
  if (occ) {
    const long long c = base[blockIdx.x] + sh[threadIdx.x] - 1;
    cidx[v] = (int)c;
    vox[c] = (int)v;
  } else {
    cidx[v] = -1;
  }
}

void build_compact_map(dda_problem *p) {
  const long long nb = (p->N + kMapBlock - 1) / kMapBlock;
  int *cnt = nullptr;
  long long *base = nullptr;
  HIPCHK(hipMalloc(&cnt, sizeof(int) * nb));
  HIPCHK(hipMalloc(&base, sizeof(long long) * nb));
  try {
    hipLaunchKernelGGL(k_map_count, dim3((unsigned)nb), dim3(kMapBlock), 0, p->st, p->mask, p->N, cnt);
    HIPCHK(hipGetLastError());
    std::vector<int> hc(nb);
    std::vector<long long> hb(nb);
    HIPCHK(hipMemcpyAsync(hc.data(), cnt, sizeof(int) * nb, hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));
    long long acc = 0;
    for (long long b = 0; b < nb; ++b) {
      hb[b] = acc;
      acc += hc[b];
    }
    REQUIRE(acc == p->nocc, DDA_EDEVICE, "occupied-voxel count mismatch (%lld vs %lld)", acc, p->nocc);
    HIPCHK(hipMalloc(&p->cidx, sizeof(int) * p->N));
    HIPCHK(hipMalloc(&p->vox, sizeof(int) * p->nocc));
    HIPCHK(hipMemcpyAsync(base, hb.data(), sizeof(long long) * nb, hipMemcpyHostToDevice, p->st));
    hipLaunchKernelGGL(k_map_fill, dim3((unsigned)nb), dim3(kMapBlock), 0, p->st, p->mask, p->N,
                       base, p->cidx, p->vox);
    HIPCHK(hipGetLastError());
    // the first and last entries (voxel order, z slowest) bound the occupied z layers
    int ends[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(&ends[0], p->vox, sizeof(int), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipMemcpyAsync(&ends[1], p->vox + (p->nocc - 1), sizeof(int), hipMemcpyDeviceToHost, p->st));
    HIPCHK(hipStreamSynchronize(p->st));  // hb and ends are host-local
    const long long plane = (long long)p->nx * p->ny;
    p->pz0 = (int)(ends[0] / plane);
    p->pbz = (int)(ends[1] / plane) - p->pz0 + 1;
  } catch (...) {
    (void)hipFree(cnt);
    (void)hipFree(base);
    throw;
  }
  HIPCHK(hipFree(cnt));
  HIPCHK(hipFree(base));
}

// Caller's box <-> compact, through the frame rotation: gather out[r][a][c] =
// in[r][a'][vox'[c]] (a' the caller's component of a, vox' the caller's voxel of entry c);
// scatter, over the caller's voxels e, out[r][a][e] = in[r][a_int][cidx[v(e)]] on occupied
// voxels and, in air, fill[r][a][e] (or 0 without fill).
__global__ void k_gather(const double2 *in, const int *vox, long long N, long long nocc, Frame fr,
                         double2 *out) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y / 3, a = blockIdx.y % 3;
  if (c >= nocc) return;
  out[(long long)blockIdx.y * nocc + c] = in[((long long)r * 3 + fr.comp_ext(a)) * N + fr.to_ext(vox[c])];
}

__global__ void k_scatter(const double2 *in, const int *cidx, long long N, long long nocc, Frame fr,
                          const double2 *fill, double2 *out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y / 3, a = blockIdx.y % 3;
  if (e >= N) return;
  const int c = cidx[fr.to_int(e)];
  const long long o = (long long)blockIdx.y * N + e;
  out[o] = c >= 0 ? in[((long long)r * 3 + fr.comp_int(a)) * nocc + c]
                  : (fill ? fill[o] : make_double2(0.0, 0.0));
}

void to_compact(dda_problem *p, int nrhs, const double2 *box, double2 *comp) {
  hipLaunchKernelGGL(k_gather, dim3(nblk(p->nocc, 256), 3 * nrhs), dim3(256), 0, p->st, box, p->vox,
                     p->N, p->nocc, p->fr, comp);
  HIPCHK(hipGetLastError());
}

void to_box(dda_problem *p, int nrhs, const double2 *comp, const double2 *fill, double2 *box) {
  hipLaunchKernelGGL(k_scatter, dim3(nblk(p->N, 256), 3 * nrhs), dim3(256), 0, p->st, comp, p->cidx,
                     p->N, p->nocc, p->fr, fill, box);
  HIPCHK(hipGetLastError());
}

// Internal copies of the caller's mask and permittivity in the rotated frame.
__global__ void k_to_frame(const uint8_t *mask, const double2 *eps, long long N, Frame fr,
                           uint8_t *mask_out, double2 *eps_out) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const long long e = fr.to_ext(v);
  mask_out[v] = mask[e];
  eps_out[v] = eps[e];
}

void copy_to_frame(dda_problem *p, const uint8_t *mask, const double2 *eps) {
  hipLaunchKernelGGL(k_to_frame, dim3(nblk(p->N, 256)), dim3(256), 0, p->st, mask, eps, p->N, p->fr,
                     p->mask, p->eps);
  HIPCHK(hipGetLastError());
}


void setup_alpha(dda_problem *p, int nrhs, const double *S_host) {
  HIPCHK(hipMemcpyAsync(p->Sdev, S_host, sizeof(double) * nrhs, hipMemcpyHostToDevice, p->st));
  KTimer t(&p->prof, p->st, "alpha_setup", 33.0 * p->N * nrhs);
  hipLaunchKernelGGL(k_alpha, dim3(nblk(p->N, 256), nrhs), dim3(256), 0, p->st, p->mask, p->eps,
                     p->N, p->k * p->d, p->Sdev, p->ainv);
  HIPCHK(hipGetLastError());
}

void setup_rhs(dda_problem *p, int nrhs, const double *dir, const double *pol, double2 *b,
               int conjugate) {
  std::vector<double> dp(6 * nrhs);
  for (int r = 0; r < nrhs; ++r)
    for (int a = 0; a < 3; ++a) {
      dp[6 * r + a] = dir[3 * r + a];
      dp[6 * r + 3 + a] = pol[3 * r + a];
    }
  double *dd = p->dscal + 8 * p->R;  // scratch area after the per-RHS scalars
  HIPCHK(hipMemcpyAsync(dd, dp.data(), sizeof(double) * 6 * nrhs, hipMemcpyHostToDevice, p->st));
  KTimer t(&p->prof, p->st, "incident_field", 52.0 * p->nocc * nrhs);
  hipLaunchKernelGGL(k_incident, dim3(nblk(p->nocc, 256), nrhs), dim3(256), 0, p->st, p->vox,
                     p->nocc, p->nx, p->ny, p->nz, p->k, p->d, dd, conjugate, b);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(p->st));  // dp is host-local
}

// The padded kernel's 3-D spectrum, kept as octants: FP64 and FP32 for the product, and its
// imaginary part (the spectrum of d^3 Im G) for the scattering sum.
static void kernel_spectrum(dda_problem *p) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const long long L3 = 8LL * p->N;
  double2 *tmp = nullptr;
  HIPCHK(hipMalloc(&tmp, sizeof(double2) * 6 * L3));
  try {
    hipLaunchKernelGGL(k_green_pad, dim3(nblk(L3, 256)), dim3(256), 0, p->st, tmp, nx, ny, nz, p->k,
                       p->d);
    HIPCHK(hipGetLastError());
    fft_rows_plain(p, p->px, tmp, 6LL * (2 * nz) * (2 * ny), 0);
    fft_strided_plain(p, p->py, tmp, 6LL * (2 * nz), 2LL * nx, 0);
    fft_strided_plain(p, p->pz, tmp, 6LL, 4LL * nx * ny, 0);
    extract_octant(p, tmp, p->khat64);
    extract_octant(p, tmp, p->khat32);
    extract_octant<double2, true>(p, tmp, p->khatI64);
    HIPCHK(hipStreamSynchronize(p->st));
  } catch (...) {
    (void)hipFree(tmp);
    throw;
  }
  HIPCHK(hipFree(tmp));
}

template <typename T> static void zpass_autotune(dda_problem *p, const cplx<T> *khat);
template <typename T>
static void op_passes(dda_problem *p, int nrhs, const double2 *x, double2 *y,
                      const cplx<T> *khat, const double *xscale, int kind);

void operator_setup(dda_problem *p) {
  // validation, mean permittivity and the compact index map
  const int nb = 1024;
  double *part = nullptr;
  HIPCHK(hipMalloc(&part, sizeof(double) * 6 * nb));
  hipLaunchKernelGGL(k_validate, dim3(nb), dim3(256), 0, p->st, p->mask, p->eps, p->N, part);
  std::vector<double> h(6 * nb);
  hipError_t e1 = hipGetLastError();
  hipError_t e2 = hipMemcpyAsync(h.data(), part, sizeof(double) * 6 * nb, hipMemcpyDeviceToHost, p->st);
  hipError_t e3 = hipStreamSynchronize(p->st);
  (void)hipFree(part);
  REQUIRE(e1 == hipSuccess && e2 == hipSuccess && e3 == hipSuccess, DDA_EDEVICE,
          "validation kernel failed: %s", hipGetErrorString(e1 != hipSuccess ? e1 : (e2 != hipSuccess ? e2 : e3)));
  double occ = 0, bad = 0, sr = 0, si = 0, qr = 0, qi = 0;
  for (int b = 0; b < nb; ++b) {
    occ += h[6 * b];
    bad += h[6 * b + 1];
    sr += h[6 * b + 2];
    si += h[6 * b + 3];
    qr += h[6 * b + 4];
    qi += h[6 * b + 5];
  }
  REQUIRE(occ > 0, DDA_EINVAL, "the mask has no occupied voxel");
  REQUIRE(bad == 0, DDA_EINVAL,
          "%.0f occupied voxel(s) have eps = 1, eps = -2 or a non-finite eps (polarisability undefined)",
          bad);
  p->n_occ = (long long)occ;
  p->nocc = p->n_occ;
  p->eps_mean = make_double2(sr / occ, si / occ);
  p->cm_mean = make_double2(qr / occ, qi / occ);
  build_compact_map(p);
}

// Kernel spectra (FP64, FP32) and the z-pass tile widths.
void operator_spectrum_setup(dda_problem *p) {
  const long long oct = 6LL * (p->nx + 1) * (p->ny + 1) * (p->nz + 1);
  const int nzz = 2 * p->nz;
  int G = 0, P = 0;
  p->zreg = zmr_split(nzz, &G, &P) ? 1 : 0;
  HIPCHK(hipMalloc(&p->khat64, sizeof(double2) * oct));
  HIPCHK(hipMalloc(&p->khat32, sizeof(float2) * oct));
  // the Im G spectrum of the scattering sum, so that no later call allocates
  HIPCHK(hipMalloc(&p->khatI64, sizeof(double2) * oct));
  kernel_spectrum(p);
  zpass_autotune<double>(p, p->khat64);
  zpass_autotune<float>(p, p->khat32);
  // x / y pass shapes of the operator, on the zero Krylov basis, in the precision the Krylov
  // iterations run in (FP32 refinement applies the FP64 product only for its few outer
  // residuals, which keep the launch rule's shapes)
  const int nt = std::min(p->R, 8);
  if (p->opt.precision == 1)
    fft_tile_autotune(p, FP_OP_X_FWD, 1, nt,
                      [&] { op_passes<float>(p, nt, p->V, p->work, p->khat32, nullptr, 0); });
  else
    fft_tile_autotune(p, FP_OP_X_FWD, 0, nt,
                      [&] { op_passes<double>(p, nt, p->V, p->work, p->khat64, nullptr, 0); });
}

// ----------------------------------------------------------------------------- the product

// Items per workgroup of the register z pass: the most (a power of two up to 16) that still
// leaves at least 2048 workgroups (8 per CU).  More items per workgroup stage the spectrum
// slab fewer times and overlap more loads with arithmetic; measured at 128^3 (2 RHS) and at
// 40^3 - 96^3 (32 RHS), this choice is within 5 % of the best fixed one.
static int zpass_ipw(long long tiles, int nrhs) {
  int ipw = 1;
  while (ipw * 2 <= std::min(16, 4 * nrhs) &&
         tiles * ((4LL * nrhs + 2 * ipw - 1) / (2 * ipw)) >= 2048)
    ipw *= 2;
  return ipw;
}

// Launch the fused z pass with `tw` columns per tile (a power of two; 0: the autotuned choice)
// and, for the register z pass, `ipw` items per workgroup (0: zpass_ipw, or the forced value).
template <typename T>
static void zpass(dda_problem *p, int nrhs, cplx<T> *w1, const cplx<T> *khat, int tw = 0,
                  bool timed = true, int ipw = 0) {
  const int n = p->pz.n;
  const double sz = sizeof(cplx<T>);
  const double bytes = nrhs * (2.0 * 3.0 * 4.0 * p->nx * p->ny * p->nz * sz) +
                       6.0 * (p->nx + 1) * (p->ny + 1) * (p->nz + 1) * sz;
  if (tw <= 0) tw = p->ztw[sizeof(T) == 8 ? 0 : 1];
  if (tw <= 0) tw = 1;
  if (ipw <= 0) ipw = p->zipw[sizeof(T) == 8 ? 0 : 1];
  KTimer t(timed ? &p->prof : nullptr, p->st, sizeof(T) == 8 ? "zpass_f64" : "zpass_f32", bytes);
  if (p->zreg) {
    ZRArgs a;
    a.nx = p->nx;
    a.ny = p->ny;
    a.nz = p->nz;
    a.plane = p->zplane;
    a.tw = tw;
    a.tiles_x = (p->nx + 1 + tw - 1) / tw;
    a.nrhs = nrhs;
    if (ipw <= 0) ipw = zpass_ipw((long long)a.tiles_x * (p->ny + 1), nrhs);
    a.ipw = std::min(ipw, 4 * nrhs);
    a.nch = (4 * nrhs + a.ipw - 1) / a.ipw;
    a.nblk = (long long)a.tiles_x * (p->ny + 1) * a.nch;
    a.act = p->act;
    int G = 0, P = 0;
    zmr_split(n, &G, &P);
    zmr_launch<T>(n, (unsigned)xcd_grid(a.nblk), 3 * tw * zmr_tpc(G, P), zmr_lds<T>(G, P, tw, p->nz),
                  p->st, w1, tw_of<T>(p->pz), khat, a);
    HIPCHK(hipGetLastError());
    return;
  }
  constexpr int EPT = EptOf<T>::value;
  ZArgs a;
  a.pl = desc(p->pz);
  a.nz = p->nz;
  a.ny = p->ny;
  a.nx = p->nx;
  a.plane = 4LL * p->nx * p->ny;
  a.zstride = p->zplane;
  a.tw = tw;
  a.twsh = ilog2_exact(tw);
  a.ntiles = (a.plane + tw - 1) / tw;
  a.nrhs = nrhs;
  a.act = p->act;
  const int threads = 3 * tw * tpc_of(n);
  const size_t lds = (size_t)lds_elems(n, 3 * tw + 1) * sizeof(cplx<T>);
  with_static_n(n, [&](auto nf) {
    auto fn = k_zpass<T, EPT, decltype(nf)::value>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3((unsigned)xcd_grid(a.ntiles * nrhs)), dim3(threads), lds, p->st,
                       w1, tw_of<T>(p->pz), khat, a);
  });
  HIPCHK(hipGetLastError());
}

// Largest power-of-two tile width that fits the LDS budget, the thread limit and the plane.
template <typename T> static int zpass_max_tw(dda_problem *p) {
  const int n = p->pz.n;
  int tw = 1;
  if (p->zreg) {
    int G = 0, P = 0;
    zmr_split(n, &G, &P);
    while (true) {
      const int t2 = tw * 2;
      if (zmr_lds<T>(G, P, t2, p->nz) > 80 * 1024 || 3 * t2 * zmr_tpc(G, P) > 256 || t2 > p->nx + 1)
        break;
      tw = t2;
    }
    return tw;
  }
  const size_t budget = std::min<size_t>(p->lds_zpass, p->lds_max);
  while (true) {
    const int t2 = tw * 2;
    if ((size_t)lds_elems(n, 3 * t2 + 1) * sizeof(cplx<T>) > budget) break;
    if (3 * t2 * tpc_of(n) > 768) break;
    if (t2 > 4LL * p->nx * p->ny) break;
    tw = t2;
  }
  return tw;
}

// Time each power-of-two tile width on the problem's own grid at min(max_rhs, 8) right-hand
// sides (the best width shifts with the RHS count) and keep the fastest.  Widths already measured in this process, per (device, grid,
// RHS count, precision), are reused: problems of a shape seen before skip the timing runs.
// The environment variable DDA_ZPASS_FORCE="tw,ipw" replaces the width and the items per
// workgroup (for tests and benchmarks of the z pass itself).
static std::mutex g_ztw_mu;
static std::map<std::tuple<int, int, int, int, int, int>, int> g_ztw;

template <typename T> static void zpass_autotune(dda_problem *p, const cplx<T> *khat) {
  const int pi = sizeof(T) == 8 ? 0 : 1;
  const int nt = std::min(p->R, 8);
  const int tmax = zpass_max_tw<T>(p);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  const auto key = std::make_tuple(dev, p->nx, p->ny, p->nz, nt, (int)sizeof(T));
  bool cached = false;
  {
    std::lock_guard<std::mutex> lk(g_ztw_mu);
    const auto it = g_ztw.find(key);
    if (it != g_ztw.end()) {
      p->ztw[pi] = it->second;
      cached = true;
    }
  }
  if (!cached) {
    cplx<T> *w1 = reinterpret_cast<cplx<T> *>(p->w1);
    HIPCHK(hipMemsetAsync(w1, 0, sizeof(cplx<T>) * nt * 3 * p->nz * p->zplane, p->st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    int best_tw = tmax;
    for (int tw = tmax; tw >= 1; tw /= 2) {
      zpass<T>(p, nt, w1, khat, tw, false);  // warm
      HIPCHK(hipEventRecord(e0, p->st));
      for (int rep = 0; rep < 3; ++rep) zpass<T>(p, nt, w1, khat, tw, false);
      HIPCHK(hipEventRecord(e1, p->st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best * 0.97f) {
        best = ms;
        best_tw = tw;
      }
      if (tw <= (p->zreg ? 1 : 2)) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->ztw[pi] = best_tw;
    std::lock_guard<std::mutex> lk(g_ztw_mu);
    g_ztw[key] = best_tw;
  }
  if (const char *f = getenv("DDA_ZPASS_FORCE")) {
    int tw = 0, ipw = 0;
    REQUIRE(sscanf(f, "%d,%d", &tw, &ipw) == 2 && tw >= 1 && tw <= tmax && (tw & (tw - 1)) == 0 &&
                ipw >= 1,
            DDA_EINVAL, "DDA_ZPASS_FORCE=\"%s\": want \"tw,ipw\" with tw a power of two <= %d and ipw >= 1",
            f, tmax);
    p->ztw[pi] = tw;
    p->zipw[pi] = ipw;
  }
}

// kind 0: DDA operator; kind 1: Im G convolution (scattering sum)
template <typename T>
static void op_passes(dda_problem *p, int nrhs, const double2 *x, double2 *y,
                      const cplx<T> *khat, const double *xscale, int kind) {
  const int nx = p->nx, ny = p->ny, nz = p->nz;
  const double sz = sizeof(cplx<T>);
  cplx<T> *w0 = reinterpret_cast<cplx<T> *>(p->w0);
  cplx<T> *w1 = reinterpret_cast<cplx<T> *>(p->w1);
  const long long rows = (long long)nrhs * 3 * nz * ny;
  const double fsuf = sizeof(T) == 8 ? 0 : 1;
  (void)fsuf;
  // P1: x rows (masked) -> zero-padded length-2nx FFT
  {
    RowArgs a{};
    a.rows = rows;
    a.n_in = nx;
    a.n_out = 2 * nx;
    a.in_stride = nx;
    a.out_stride = 2 * nx;
    a.sign = -1;
    a.cidx = p->cidx;
    a.nocc = p->nocc;
    a.vox_rows = (long long)nz * ny;
    a.rhs_rows = 3LL * nz * ny;
    a.nx = nx;
    a.N = p->N;
    a.xscale = xscale;
    launch_rows<T, ROW_OP_FWD, double2, cplx<T>>(
        p, p->px, x, w0, a, sizeof(T) == 8 ? "op_x_fwd_f64" : "op_x_fwd_f32",
        rows * (4.0 * nx + sz * 2 * nx) + nrhs * 48.0 * p->nocc, FP_OP_X_FWD);
  }
  // P2: y transform, ny rows zero-padded to 2ny
  launch_strided<T>(p, p->py, w0, w1, (long long)nrhs * 3 * nz, 2LL * nx, ny, 2 * ny,
                    (long long)ny * 2 * nx, p->zplane, -1,
                    sizeof(T) == 8 ? "op_y_fwd_f64" : "op_y_fwd_f32",
                    nrhs * 3.0 * nz * 2 * nx * (ny + 2.0 * ny) * sz, 3LL * nz, FP_OP_Y_FWD);
  // P3: z transform, kernel multiply, inverse z transform (in place)
  if (!p->tune_xy) zpass<T>(p, nrhs, w1, khat);
  // P4: inverse y transform, keep ny rows
  launch_strided<T>(p, p->py, w1, w0, (long long)nrhs * 3 * nz, 2LL * nx, 2 * ny, ny,
                    p->zplane, (long long)ny * 2 * nx, +1,
                    sizeof(T) == 8 ? "op_y_inv_f64" : "op_y_inv_f32",
                    nrhs * 3.0 * nz * 2 * nx * (2.0 * ny + ny) * sz, 3LL * nz, FP_OP_Y_INV);
  // P5: inverse x transform, keep nx, diagonal and mask epilogue
  {
    RowArgs a{};
    a.rows = rows;
    a.n_in = 2 * nx;
    a.n_out = nx;
    a.in_stride = 2 * nx;
    a.out_stride = nx;
    a.sign = +1;
    a.cidx = p->cidx;
    a.nocc = p->nocc;
    a.vox_rows = (long long)nz * ny;
    a.rhs_rows = 3LL * nz * ny;
    a.nx = nx;
    a.N = p->N;
    a.ainv = p->ainv;
    a.xin = x;
    a.xscale = xscale;
    a.scale = 1.0 / (8.0 * (double)p->N);
    if (kind == 0)
      launch_rows<T, ROW_OP_INV, cplx<T>, double2>(
          p, p->px, w0, y, a, sizeof(T) == 8 ? "op_x_inv_f64" : "op_x_inv_f32",
          rows * (sz * 2 * nx + 4.0 * nx) + nrhs * (96.0 * p->nocc + 16.0 * p->N), FP_OP_X_INV);
    else
      launch_rows<T, ROW_IMG_INV, cplx<T>, double2>(p, p->px, w0, y, a, "imag_x_inv",
                                                    rows * (sz * 2 * nx + 4.0 * nx) + nrhs * 48.0 * p->nocc);
  }
}

void apply_operator(dda_problem *p, int nrhs, const double2 *x, double2 *y, int fp32,
                    const double *xscale) {
  if (fp32)
    op_passes<float>(p, nrhs, x, y, p->khat32, xscale, 0);
  else
    op_passes<double>(p, nrhs, x, y, p->khat64, xscale, 0);
}

void apply_imag_conv(dda_problem *p, int nrhs, const double2 *x, double2 *y) {
  op_passes<double>(p, nrhs, x, y, p->khatI64, nullptr, 1);
}

}  // namespace dda
