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
