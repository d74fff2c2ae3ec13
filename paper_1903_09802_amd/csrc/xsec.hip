// Cross sections of a solved dipole array and the adjoint gradient of C_ext (compact
// field vectors, see the problem handle).
//
// With the paper's scaling (polarisation density c, voxel volume omitted from alpha,
// Sec. 2.1) the Draine-Flatau expressions become, for |E_0| = 1,
//   C_ext = 4 pi k d^3 sum Im(E_inc^* . c)
//   C_abs = 4 pi k d^3 sum |c|^2 (-Im alpha^{-1} - (2/3)(k d)^3)
//   C_sca = 4 pi k d^3 [(2/3)(k d)^3 sum |c|^2 + sum_{i != j} c_i^H (d^3 Im G_ij) c_j],
// the last double sum applied as an FFT convolution with the Im G kernel.
// Gradient: with A lambda = conj(E_inc) (A = A^T), h'_j = -(d alpha_j^{-1}/d eps_j)
// sum_a lambda_ja c_ja and dC_ext/dRe eps + i dC_ext/dIm eps = 4 pi k d^3 i conj(h'_j).
#include <cmath>

#include "common.h"

namespace dda {

// partial[(r * B + blk) * 4 + q]: q = 0 ext, 1 abs weight sum, 2 Re(c^H u), 3 |c|^2.
// c, E, u compact [R][3][nocc]; ainv per voxel [R][N].
__global__ void k_xsec_partial(const double2 *c, const double2 *E, const double2 *u,
                               const double2 *ainv, const int *vox, long long N, long long nocc,
                               double kd, double *partial, int B) {
  const int r = blockIdx.y;
  __shared__ double sh[4][256];
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  const double rr = (2.0 / 3.0) * kd * kd * kd;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nocc;
       q += (long long)gridDim.x * blockDim.x) {
    const double2 ai = ainv[r * N + vox[q]];
    double c2 = 0;
    for (int a = 0; a < 3; ++a) {
      const long long o = ((long long)r * 3 + a) * nocc + q;
      const double2 cv = c[o];
      const double2 ev = E[o];
      s0 += ev.x * cv.y - ev.y * cv.x;  // Im(conj(E) c)
      if (u) {
        const double2 uv = u[o];
        s2 += cv.x * uv.x + cv.y * uv.y;  // Re(conj(c) u)
      }
      c2 += cv.x * cv.x + cv.y * cv.y;
    }
    s1 += c2 * (-ai.y - rr);
    s3 += c2;
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = s2;
  sh[3][threadIdx.x] = s3;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int q = 0; q < 4; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) partial[((long long)r * B + blockIdx.x) * 4 + q] = sh[q][0];
}

void cross_sections(dda_problem *p, int nrhs, const double *dir, const double *pol,
                    const double2 *c, double *cext, double *cabs, double *csca) {
  const long long N = p->N;
  const int B = 512;
  setup_rhs(p, nrhs, dir, pol, p->work2, 0);
  const double2 *u = nullptr;
  if (csca) {
    apply_imag_conv(p, nrhs, c, p->work);
    u = p->work;
  }
  double *part = p->partial;  // [nrhs][B][4] fits the reduction buffer
  REQUIRE((size_t)nrhs * B * 4 <= p->partial_elems, DDA_EINVAL, "reduction buffer too small");
  {
    KTimer t(&p->prof, p->st, "xsec_reduce", (double)nrhs * p->nocc * (16.0 * 10 + 4.0));
    hipLaunchKernelGGL(k_xsec_partial, dim3(B, nrhs), dim3(256), 0, p->st, c, p->work2, u, p->ainv,
                       p->vox, N, p->nocc, p->k * p->d, part, B);
    HIPCHK(hipGetLastError());
  }
  std::vector<double> h((size_t)nrhs * B * 4);
  HIPCHK(hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  const double kd = p->k * p->d;
  const double pref = 4.0 * DDA_PI * p->k * p->d * p->d * p->d;
  for (int r = 0; r < nrhs; ++r) {
    double s[4] = {0, 0, 0, 0};
    for (int b = 0; b < B; ++b)
      for (int q = 0; q < 4; ++q) s[q] += h[((size_t)r * B + b) * 4 + q];
    if (cext) cext[r] = pref * s[0];
    if (cabs) cabs[r] = pref * s[1];
    if (csca) csca[r] = pref * ((2.0 / 3.0) * kd * kd * kd * s[3] + s[2]);
  }
}

// c, lam compact [3][nocc]; grad per voxel [N] in the caller's layout, zero in air.
__global__ void k_grad(const double2 *c, const double2 *lam, const double2 *eps, const int *cidx,
                       long long N, long long nocc, Frame fr, double kd, double S, double pref,
                       double2 *grad) {
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= N) return;
  const int q = cidx[v];
  const long long ve = fr.to_ext(v);
  if (q < 0) {
    grad[ve] = make_double2(0.0, 0.0);
    return;
  }
  double2 acc = make_double2(0.0, 0.0);
  for (int a = 0; a < 3; ++a) acc = cadd(acc, cmul(lam[a * nocc + q], c[a * nocc + q]));
  const double2 da = ldr_dalpha_inv(eps[v], kd, S);
  const double2 hp = make_double2(-(da.x * acc.x - da.y * acc.y), -(da.x * acc.y + da.y * acc.x));
  // i * conj(h') = (Im h', Re h')
  grad[ve] = make_double2(pref * hp.y, pref * hp.x);
}

void grad_kernel(dda_problem *p, const double2 *c, const double2 *lam, double S, double2 *grad) {
  KTimer t(&p->prof, p->st, "adjoint_grad", 113.0 * p->N);
  hipLaunchKernelGGL(k_grad, dim3((unsigned)((p->N + 255) / 256)), dim3(256), 0, p->st, c, lam,
                     p->eps, p->cidx, p->N, p->nocc, p->fr, p->k * p->d, S,
                     4.0 * DDA_PI * p->k * p->d * p->d * p->d, grad);
  HIPCHK(hipGetLastError());
}

}  // namespace dda

// ----------------------------------------------------------------------------- allocation-free

// dda_cross_sections_noalloc: C_ext and C_abs with every scratch byte in one static device
// array per GPU (no allocation on the device or the host, no exception).  The array holds the
// per-block partial sums [nrhs][kXsBlocks][2] and the scaled totals [2][nrhs]; every call
// overwrites all of what it reads, so nothing is cleared between calls, and calls that overlap
// on one GPU (other streams or threads) race on it.
namespace dda {

constexpr int kXsBlocks = 512;
constexpr size_t kScratchDoubles = (size_t)kNoallocMaxRhs * kXsBlocks * 2 + 2 * kNoallocMaxRhs;
static __device__ __align__(256) double scratch[kScratchDoubles];

// The array's device address, one per GPU, resolved once with that GPU current.
static constexpr int kMaxDevices = 64;
static double *g_scratch_addr[kMaxDevices] = {nullptr};

hipError_t noalloc_scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (__atomic_load_n(&g_scratch_addr[dev], __ATOMIC_ACQUIRE)) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  __atomic_store_n(&g_scratch_addr[dev], static_cast<double *>(ptr), __ATOMIC_RELEASE);
  return hipSuccess;
}

struct XsWaves {
  int nrhs;
  double dir[kNoallocMaxRhs][3], pol[kNoallocMaxRhs][3], S[kNoallocMaxRhs];  // library frame
};

// Per block: sum over its compact entries q of Im(conj(E) . c) and |c|^2 (-Im alpha^{-1} -
// (2/3)(k d)^3), with c read from the caller's box layout through the frame, E^inc and 1/alpha
// computed in place.  part[(r * kXsBlocks + block) * 2 + {0, 1}].
__global__ void __launch_bounds__(256) k_xsec_box(const double2 *cbox, const int *vox,
                                                  const double2 *eps, long long N, long long nocc,
                                                  Frame fr, double k, double d, XsWaves wv,
                                                  double *part) {
  const int r = blockIdx.y;
  __shared__ double sh[2][256];
  const double kd = k * d, rr = (2.0 / 3.0) * kd * kd * kd;
  double s0 = 0.0, s1 = 0.0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < nocc;
       q += (long long)gridDim.x * blockDim.x) {
    const long long v = vox[q];
    const int ix = (int)(v % fr.nx), iy = (int)((v / fr.nx) % fr.ny),
              iz = (int)(v / ((long long)fr.nx * fr.ny));
    const double x = (ix - 0.5 * (fr.nx - 1)) * d, y = (iy - 0.5 * (fr.ny - 1)) * d,
                 z = (iz - 0.5 * (fr.nz - 1)) * d;
    double sn, cs;
    sincos(k * (wv.dir[r][0] * x + wv.dir[r][1] * y + wv.dir[r][2] * z), &sn, &cs);
    const long long e = fr.to_ext(v);
    double c2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double2 cv = cbox[((long long)r * 3 + fr.comp_ext(a)) * N + e];
      const double2 ev = make_double2(wv.pol[r][a] * cs, wv.pol[r][a] * sn);
      s0 += ev.x * cv.y - ev.y * cv.x;
      c2 += cv.x * cv.x + cv.y * cv.y;
    }
    s1 += c2 * (-ldr_alpha_inv(eps[v], kd, wv.S[r]).y - rr);
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[((long long)r * kXsBlocks + blockIdx.x) * 2 + 0] = sh[0][0];
    part[((long long)r * kXsBlocks + blockIdx.x) * 2 + 1] = sh[1][0];
  }
}

// tot[q * nrhs + r] = pref * sum over the blocks of part (block order fixed); one block per r.
__global__ void __launch_bounds__(256) k_xsec_total(const double *part, double pref, int nrhs,
                                                    double *tot) {
  const int r = blockIdx.x;
  __shared__ double sh[2][256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < kXsBlocks; i += blockDim.x) {
    a += part[((long long)r * kXsBlocks + i) * 2 + 0];
    b += part[((long long)r * kXsBlocks + i) * 2 + 1];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    tot[r] = pref * sh[0][0];
    tot[nrhs + r] = pref * sh[1][0];
  }
}

}  // namespace dda

extern "C" dda_status dda_cross_sections_noalloc(dda_problem *p, int nrhs, const double *dir_host,
                                                 const double *pol_host, const double *c_dev,
                                                 double *cext, double *cabs) {
  using namespace dda;
  auto fail = [](dda_status st, const char *msg) {
    set_error("%s", msg);
    return st;
  };
  set_error("%s", "");
  if (!p) return fail(DDA_EINVAL, "problem is NULL");
  if (nrhs < 1 || nrhs > kNoallocMaxRhs || nrhs > p->R)
    return fail(DDA_EINVAL, "dda_cross_sections_noalloc: nrhs must be in [1, min(max_rhs, 16)] "
                            "(its static scratch holds 16 waves)");
  if (!c_dev || !dir_host || !pol_host) return fail(DDA_EINVAL, "c_dev, dir_host and pol_host are required");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != p->dev)
    return fail(DDA_EDEVICE, "dda_cross_sections_noalloc: the handle's device is not current");
  double *base = dev < kMaxDevices ? __atomic_load_n(&g_scratch_addr[dev], __ATOMIC_ACQUIRE) : nullptr;
  if (!base) return fail(DDA_ESTATE, "static scratch address not resolved on this device");
  XsWaves wv;
  wv.nrhs = nrhs;
  for (int r = 0; r < nrhs; ++r) {
    const double *dv = dir_host + 3 * r, *ev = pol_host + 3 * r;
    const double nd = std::sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const double ne = std::sqrt(ev[0] * ev[0] + ev[1] * ev[1] + ev[2] * ev[2]);
    const double de = dv[0] * ev[0] + dv[1] * ev[1] + dv[2] * ev[2];
    if (!(std::fabs(nd - 1.0) <= 1e-9 && std::fabs(ne - 1.0) <= 1e-9 && std::fabs(de) <= 1e-9))
      return fail(DDA_EINVAL, "direction and polarisation must be orthogonal unit vectors");
    double S = 0.0;
    for (int a = 0; a < 3; ++a) {
      S += (dv[a] * ev[a]) * (dv[a] * ev[a]);
      wv.dir[r][a] = dv[p->fr.comp_ext(a)];
      wv.pol[r][a] = ev[p->fr.comp_ext(a)];
    }
    wv.S[r] = S;
  }
  double *part = base;
  double *tot = base + (size_t)kNoallocMaxRhs * kXsBlocks * 2;
  hipLaunchKernelGGL(k_xsec_box, dim3(kXsBlocks, nrhs), dim3(256), 0, p->st,
                     reinterpret_cast<const double2 *>(c_dev), p->vox, p->eps, p->N, p->nocc,
                     p->fr, p->k, p->d, wv, part);
  const double pref = 4.0 * DDA_PI * p->k * p->d * p->d * p->d;
  hipLaunchKernelGGL(k_xsec_total, dim3(nrhs), dim3(256), 0, p->st, part, pref, nrhs, tot);
  double host[2 * kNoallocMaxRhs];
  hipError_t e = hipGetLastError();
  if (e == hipSuccess)
    e = hipMemcpyAsync(host, tot, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, p->st);
  if (e == hipSuccess) e = hipStreamSynchronize(p->st);
  if (e != hipSuccess) {
    set_error("dda_cross_sections_noalloc: %s", hipGetErrorString(e));
    return DDA_EDEVICE;
  }
  for (int r = 0; r < nrhs; ++r) {
    if (cext) cext[r] = host[r];
    if (cabs) cabs[r] = host[nrhs + r];
  }
  return DDA_OK;
}
