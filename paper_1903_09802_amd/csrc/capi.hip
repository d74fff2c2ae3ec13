// C-ABI of the DDA library: argument checking, allocation, and the calls of include/dda.h.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include <cstdlib>

#include "common.h"

using namespace dda;

namespace {

template <typename F> dda_status guarded(F &&f) {
  try {
    set_error("%s", "");
    return f();
  } catch (const Fail &e) {
    return e.st;
  } catch (const std::bad_alloc &) {
    set_error("host allocation failed");
    return DDA_ENOMEM;
  } catch (...) {
    set_error("unexpected internal error");
    return DDA_EDEVICE;
  }
}

void free_all(dda_problem *p) {
  auto F = [](void *ptr) {
    if (ptr) (void)hipFree(ptr);
  };
  F(p->mask); F(p->eps); F(p->cidx); F(p->vox); F(p->khat64); F(p->khat32); F(p->khatI64); F(p->w0); F(p->w1);
  F(p->ainv); F(p->Sdev); F(p->V); F(p->work); F(p->work2); F(p->bvec); F(p->xvec); F(p->vsc);
  F(p->H); F(p->givens); F(p->gvec); F(p->hcol); F(p->hcol2);
  F(p->ycoef); F(p->hnrm); F(p->hraw); F(p->lmat); F(p->partial); F(p->dscal); F(p->dflag);
  F(p->ctl); F(p->ones); F(p->bnrm); F(p->cres); F(p->hist); F(p->adj); F(p->stage);
  if (p->hpin) (void)hipHostFree(p->hpin);
  if (p->hlive) (void)hipHostFree(p->hlive);
  p->hpin = nullptr;
  p->hlive = nullptr;
  drop_graphs(p);
  if (p->cap_st) (void)hipStreamDestroy(p->cap_st);
  p->cap_st = nullptr;
  precond_free(p);
  plan_destroy(p->px); plan_destroy(p->py); plan_destroy(p->pz);
  plan_destroy(p->ux); plan_destroy(p->uy);
  p->prof.destroy();
}

void check_waves(int nrhs, const double *dir, const double *pol, std::vector<double> &S) {
  REQUIRE(nrhs >= 1, DDA_EINVAL, "nrhs must be >= 1");
  REQUIRE(dir && pol, DDA_EINVAL, "dir_host and pol_host are required");
  S.resize(nrhs);
  for (int r = 0; r < nrhs; ++r) {
    const double *d = dir + 3 * r, *e = pol + 3 * r;
    const double nd = std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    const double ne = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    const double de = d[0] * e[0] + d[1] * e[1] + d[2] * e[2];
    REQUIRE(std::fabs(nd - 1.0) <= 1e-9 && std::fabs(ne - 1.0) <= 1e-9 && std::fabs(de) <= 1e-9,
            DDA_EINVAL, "wave %d: direction and polarisation must be orthogonal unit vectors", r);
    double s = 0.0;
    for (int a = 0; a < 3; ++a) s += (d[a] * e[a]) * (d[a] * e[a]);
    S[r] = s;
  }
}

// A solve's stats record: counters zero, the caller's history buffer (input fields) kept.
dda_stats stats_in(const dda_stats *caller) {
  dda_stats s;
  std::memset(&s, 0, sizeof s);
  if (caller) {
    s.history = caller->history;
    s.history_cap = caller->history ? std::max(0, caller->history_cap) : 0;
  }
  return s;
}

dda_stats stats_out(const dda_problem *p, dda_stats s, double seconds) {
  s.t_setup = p->t_setup;
  s.t_build = p->prec_built ? p->t_build : 0.0;
  s.t_solve = seconds;
  return s;
}

// Wave vectors (3 per wave) in the library's rotated frame.
std::vector<double> in_frame(const dda_problem *p, int nrhs, const double *v) {
  std::vector<double> out(3 * (size_t)nrhs);
  for (int r = 0; r < nrhs; ++r)
    for (int a = 0; a < 3; ++a) out[3 * r + a] = v[3 * r + p->fr.comp_ext(a)];
  return out;
}

}  // namespace

extern "C" {

void dda_default_options(dda_options *opt) {
  if (!opt) return;
  opt->restart = 30;
  opt->max_iter = 2000;
  opt->tol = 1e-5;
  opt->precond = 2;
  opt->precision = 0;
  opt->max_rhs = 1;
  opt->solver = 0;
  opt->dense_axis = 2;
  opt->left_precond = 0;
  opt->alpha_avg = 0;
  opt->diag_steps = 0;
  opt->graph = 1;
}

const char *dda_last_error(void) { return get_error(); }

dda_status dda_lattice_factor(int nrhs, const double *dir_host, const double *pol_host,
                              double *S_host, double *S_mean) {
  return guarded([&]() -> dda_status {
    std::vector<double> S;
    check_waves(nrhs, dir_host, pol_host, S);
    double sum = 0.0;
    for (int r = 0; r < nrhs; ++r) {
      if (S_host) S_host[r] = S[r];
      sum += S[r];
    }
    if (S_mean) *S_mean = sum / nrhs;
    return DDA_OK;
  });
}

dda_status dda_create(int nx, int ny, int nz, const uint8_t *mask_dev, const double *eps_dev,
                      double k, double d, const dda_options *opt, void *stream,
                      dda_problem **out) {
  return guarded([&]() -> dda_status {
    const auto t0 = std::chrono::steady_clock::now();
    REQUIRE(out, DDA_EINVAL, "out is NULL");
    *out = nullptr;
    REQUIRE(nx >= 1 && ny >= 1 && nz >= 1, DDA_EINVAL, "grid dimensions must be >= 1 (got %d %d %d)",
            nx, ny, nz);
    REQUIRE(nx <= 512 && ny <= 512 && nz <= 512, DDA_EUNSUPPORTED,
            "grid dimensions must be <= 512 (got %d %d %d)", nx, ny, nz);
    REQUIRE(mask_dev && eps_dev, DDA_EINVAL, "mask_dev and eps_dev are required");
    REQUIRE(k > 0.0 && d > 0.0 && std::isfinite(k) && std::isfinite(d), DDA_EINVAL,
            "k and d must be positive");
    dda_options o;
    dda_default_options(&o);
    if (opt) o = *opt;
    REQUIRE(o.restart >= 1 && o.restart < kMaxM, DDA_EINVAL, "restart must be in [1, %d]", kMaxM - 1);
    REQUIRE(o.max_iter >= 1, DDA_EINVAL, "max_iter must be >= 1");
    REQUIRE(o.tol > 0.0, DDA_EINVAL, "tol must be > 0");
    REQUIRE(o.precond >= 0 && o.precond <= 2, DDA_EINVAL, "precond must be 0, 1 or 2");
    REQUIRE(o.precision == 0 || o.precision == 1, DDA_EINVAL, "precision must be 0 or 1");
    REQUIRE(o.max_rhs >= 1 && o.max_rhs <= 64, DDA_EINVAL, "max_rhs must be in [1, 64]");
    REQUIRE(o.graph == 0 || o.graph == 1, DDA_EINVAL, "graph must be 0 or 1");
    REQUIRE(o.solver == 0 || o.solver == 1, DDA_EINVAL, "solver must be 0 (GMRES) or 1 (BiCGStab)");
    REQUIRE(o.solver == 0 || o.precision == 0, DDA_EUNSUPPORTED, "BiCGStab runs in FP64 only (precision 0)");
    REQUIRE(o.solver == 0 || o.restart >= 7, DDA_EINVAL, "BiCGStab needs restart >= 7 (work vectors)");
    REQUIRE(o.dense_axis >= 0 && o.dense_axis <= 2, DDA_EINVAL, "dense_axis must be 0, 1 or 2");
    REQUIRE(o.left_precond == 0 || o.left_precond == 1, DDA_EINVAL, "left_precond must be 0 or 1");
    REQUIRE(o.left_precond == 0 || o.solver == 0, DDA_EINVAL,
            "left preconditioning is a GMRES option (solver 0)");
    REQUIRE(o.alpha_avg >= 0 && o.alpha_avg <= 2, DDA_EINVAL, "alpha_avg must be 0, 1 or 2");
    REQUIRE(o.diag_steps >= 0 && o.diag_steps <= 32, DDA_EINVAL, "diag_steps must be in [0, 32]");
    REQUIRE(o.diag_steps == 0 || o.precond != 0, DDA_EINVAL,
            "diag_steps needs a preconditioner (precond 1 or 2)");
    {
      FftPlan t;
      REQUIRE(factor_7smooth(nx, t) && factor_7smooth(ny, t) && factor_7smooth(nz, t),
              DDA_EUNSUPPORTED, "grid dimensions must factor into 2, 3, 5, 7 (got %d %d %d)", nx, ny,
              nz);
    }
    dda_problem *p = new dda_problem();
    try {
      // internal frame: the cyclic rotation of the axes that puts the dense axis last
      const int ax0 = (o.dense_axis + 1) % 3, ax1 = (o.dense_axis + 2) % 3, ax2 = o.dense_axis;
      const int ext[3] = {nx, ny, nz};
      p->fr = Frame{ext[ax0], ext[ax1], ext[ax2], nx, ny, ax0, ax1, ax2};
      nx = ext[ax0];
      ny = ext[ax1];
      nz = ext[ax2];
      p->nx = nx; p->ny = ny; p->nz = nz;
      p->N = (long long)nx * ny * nz;
      p->k = k; p->d = d;
      p->st = reinterpret_cast<hipStream_t>(stream);
      p->opt = o;
      p->R = o.max_rhs;
      int dev = 0;
      HIPCHK(hipGetDevice(&dev));
      p->dev = dev;
      HIPCHK(noalloc_scratch_init(dev));
      hipDeviceProp_t prop;
      HIPCHK(hipGetDeviceProperties(&prop, dev));
      p->lds_max = prop.sharedMemPerBlock > 0 ? (size_t)prop.sharedMemPerBlock : 65536;
      // memory estimate (bytes) before allocating
      const long long N = p->N, n3 = 3 * N, R = p->R, m = o.restart;
      double need = 0;
      need += N * 17.0;                                  // mask + eps
      need += 6.0 * (nx + 1) * (ny + 1) * (nz + 1) * 40;  // khat64 + khat32 + khatI64
      need += 8.0 * N * 6 * 16;                          // setup transient
      need += R * 3.0 * N * 2 * 16 + R * 3.0 * nz * (4.0 * nx * ny + 64) * 16;  // w0 + w1
      need += R * 16.0 * N;                              // 1 / alpha per wave
      need += R * 2.0 * kMaxM * 1024 * 16 + R * (m + 1.0) * (m + 1.0) * 16;  // reductions, Gram
      (void)n3;  // the Krylov vectors are compact: checked once the occupied voxels are counted
      size_t freeb = 0, totb = 0;
      HIPCHK(hipMemGetInfo(&freeb, &totb));
      REQUIRE(need < 0.9 * (double)freeb, DDA_ENOMEM, "problem needs about %.2f GB, %.2f GB free",
              need / 1e9, freeb / 1e9);
      plan_create(p->px, 2 * nx);
      plan_create(p->py, 2 * ny);
      plan_create(p->pz, 2 * nz);
      plan_create(p->ux, nx);
      plan_create(p->uy, ny);
      HIPCHK(hipMalloc(&p->mask, N));
      HIPCHK(hipMalloc(&p->eps, sizeof(double2) * N));
      copy_to_frame(p, mask_dev, reinterpret_cast<const double2 *>(eps_dev));
      p->w0_elems = (size_t)R * 3 * nz * ny * 2 * nx;
      // z rows of the z-pass work array are padded by 64 elements: with 4 nx ny a large power
      // of two, unpadded rows alias the same HBM channels under the z-strided access
      p->zplane = 4LL * nx * ny + 64;
      p->w1_elems = (size_t)R * 3 * nz * p->zplane;
      HIPCHK(hipMalloc(&p->w0, sizeof(double2) * p->w0_elems));
      HIPCHK(hipMalloc(&p->w1, sizeof(double2) * p->w1_elems));
      HIPCHK(hipMalloc(&p->ainv, sizeof(double2) * R * N));
      HIPCHK(hipMalloc(&p->Sdev, sizeof(double) * R));
      operator_setup(p);  // validation and the compact maps: the solver vectors are compact
      krylov_alloc(p);
      operator_spectrum_setup(p);
      HIPCHK(hipStreamSynchronize(p->st));
    } catch (...) {
      free_all(p);
      delete p;
      throw;
    }
    p->t_setup = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return DDA_OK;
  });
}

dda_status dda_build_preconditioner(dda_problem *p, double s_bar) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    REQUIRE(s_bar >= 0.0 && s_bar <= 1.0, DDA_EINVAL, "s_bar must be in [0, 1]");
    const auto t0 = std::chrono::steady_clock::now();
    drop_graphs(p);  // captured cycles read the blocks that the build replaces
    p->t_build = 0.0;
    precond_build(p, s_bar);
    if (p->prof.on) p->prof.collect();
    p->t_build = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return DDA_OK;
  });
}

dda_status dda_solve(dda_problem *p, int nrhs, const double *dir_host, const double *pol_host,
                     const double *x0_dev, double *c_dev, double *cext, double *cabs,
                     double *csca, dda_stats *stats) {
  return guarded([&]() -> dda_status {
    const auto t0 = std::chrono::steady_clock::now();
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    REQUIRE(nrhs >= 1 && nrhs <= p->R, DDA_EINVAL, "nrhs must be in [1, max_rhs = %d]", p->R);
    std::vector<double> S;
    check_waves(nrhs, dir_host, pol_host, S);
    const std::vector<double> dirs = in_frame(p, nrhs, dir_host), pols = in_frame(p, nrhs, pol_host);
    dir_host = dirs.data();
    pol_host = pols.data();
    REQUIRE(p->opt.precond == 0 || p->prec_built, DDA_ESTATE,
            "opt.precond != 0 but dda_build_preconditioner has not run");
    const long long n3 = 3 * p->nocc;
    setup_alpha(p, nrhs, S.data());
    setup_rhs(p, nrhs, dir_host, pol_host, p->bvec, 0);
    if (x0_dev)
      to_compact(p, nrhs, reinterpret_cast<const double2 *>(x0_dev), p->xvec);
    else
      HIPCHK(hipMemsetAsync(p->xvec, 0, sizeof(double2) * n3 * nrhs, p->st));
    std::vector<dda_stats> st(nrhs, stats_in(nullptr));
    if (stats)
      for (int r = 0; r < nrhs; ++r) st[r] = stats_in(&stats[r]);
    dda_status res = solve_system(p, nrhs, p->bvec, p->xvec, st.data());
    if (c_dev) to_box(p, nrhs, p->xvec, nullptr, reinterpret_cast<double2 *>(c_dev));
    if (cext || cabs || csca) cross_sections(p, nrhs, dir_host, pol_host, p->xvec, cext, cabs, csca);
    HIPCHK(hipStreamSynchronize(p->st));
    if (p->prof.on) p->prof.collect();
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats)
      for (int r = 0; r < nrhs; ++r) stats[r] = stats_out(p, st[r], sec);
    return res;
  });
}

dda_status dda_apply_operator(dda_problem *p, int nrhs, const double *dir_host,
                              const double *pol_host, const double *x_dev, double *y_dev,
                              int fp32) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    REQUIRE(nrhs >= 1 && nrhs <= p->R, DDA_EINVAL, "nrhs must be in [1, max_rhs = %d]", p->R);
    REQUIRE(x_dev && y_dev && x_dev != y_dev, DDA_EINVAL, "x_dev and y_dev must be distinct buffers");
    std::vector<double> S;
    check_waves(nrhs, dir_host, pol_host, S);
    const std::vector<double> dirs = in_frame(p, nrhs, dir_host), pols = in_frame(p, nrhs, pol_host);
    dir_host = dirs.data();
    pol_host = pols.data();
    setup_alpha(p, nrhs, S.data());
    // box -> compact, A on the occupied voxels, and y = x in air
    const double2 *xb = reinterpret_cast<const double2 *>(x_dev);
    to_compact(p, nrhs, xb, p->work2);
    apply_operator(p, nrhs, p->work2, p->work, fp32 ? 1 : 0, nullptr);
    to_box(p, nrhs, p->work, xb, reinterpret_cast<double2 *>(y_dev));
    return DDA_OK;
  });
}

dda_status dda_apply_preconditioner(dda_problem *p, int nrhs, const double *x_dev, double *y_dev,
                                    int fp32) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    REQUIRE(nrhs >= 1 && nrhs <= p->R, DDA_EINVAL, "nrhs must be in [1, max_rhs = %d]", p->R);
    REQUIRE(x_dev && y_dev, DDA_EINVAL, "x_dev and y_dev are required");
    to_compact(p, nrhs, reinterpret_cast<const double2 *>(x_dev), p->work2);
    apply_precond(p, nrhs, p->work2, p->work, fp32 ? 1 : 0, nullptr);
    to_box(p, nrhs, p->work, nullptr, reinterpret_cast<double2 *>(y_dev));
    return DDA_OK;
  });
}

dda_status dda_cross_sections(dda_problem *p, int nrhs, const double *dir_host,
                              const double *pol_host, const double *c_dev, double *cext,
                              double *cabs, double *csca) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    REQUIRE(nrhs >= 1 && nrhs <= p->R, DDA_EINVAL, "nrhs must be in [1, max_rhs = %d]", p->R);
    REQUIRE(c_dev, DDA_EINVAL, "c_dev is required");
    std::vector<double> S;
    check_waves(nrhs, dir_host, pol_host, S);
    const std::vector<double> dirs = in_frame(p, nrhs, dir_host), pols = in_frame(p, nrhs, pol_host);
    dir_host = dirs.data();
    pol_host = pols.data();
    setup_alpha(p, nrhs, S.data());
    to_compact(p, nrhs, reinterpret_cast<const double2 *>(c_dev), p->bvec);
    cross_sections(p, nrhs, dir_host, pol_host, p->bvec, cext, cabs, csca);
    if (p->prof.on) p->prof.collect();
    return DDA_OK;
  });
}

dda_status dda_grad_cext(dda_problem *p, const double *dir_host, const double *pol_host,
                         double *grad_dev, double *cext, dda_stats *stats) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    REQUIRE(grad_dev, DDA_EINVAL, "grad_dev is required");
    REQUIRE(p->opt.precond == 0 || p->prec_built, DDA_ESTATE,
            "opt.precond != 0 but dda_build_preconditioner has not run");
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<double> S;
    check_waves(1, dir_host, pol_host, S);
    const std::vector<double> dirs = in_frame(p, 1, dir_host), pols = in_frame(p, 1, pol_host);
    dir_host = dirs.data();
    pol_host = pols.data();
    const long long n3 = 3 * p->nocc;
    double2 *cfwd = p->adj;
    dda_stats st[2] = {stats_in(stats), stats_in(stats ? stats + 1 : nullptr)};
    setup_alpha(p, 1, S.data());
    // forward: A c = E_inc
    setup_rhs(p, 1, dir_host, pol_host, p->bvec, 0);
    HIPCHK(hipMemsetAsync(p->xvec, 0, sizeof(double2) * n3, p->st));
    dda_status r1 = solve_system(p, 1, p->bvec, p->xvec, &st[0]);
    HIPCHK(hipMemcpyAsync(cfwd, p->xvec, sizeof(double2) * n3, hipMemcpyDeviceToDevice, p->st));
    if (cext) cross_sections(p, 1, dir_host, pol_host, cfwd, cext, nullptr, nullptr);
    // adjoint: A lambda = conj(E_inc)
    setup_rhs(p, 1, dir_host, pol_host, p->bvec, 1);
    HIPCHK(hipMemsetAsync(p->xvec, 0, sizeof(double2) * n3, p->st));
    dda_status r2 = solve_system(p, 1, p->bvec, p->xvec, &st[1]);
    grad_kernel(p, cfwd, p->xvec, S[0], reinterpret_cast<double2 *>(grad_dev));
    HIPCHK(hipStreamSynchronize(p->st));
    const dda_status res = (r1 == DDA_OK && r2 == DDA_OK) ? DDA_OK : DDA_NOT_CONVERGED;
    if (p->prof.on) p->prof.collect();
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (stats) {
      stats[0] = stats_out(p, st[0], sec);
      stats[1] = stats_out(p, st[1], sec);
    }
    return res;
  });
}

void dda_destroy(dda_problem *p) {
  if (!p) return;
  try {
    (void)hipStreamSynchronize(p->st);
    free_all(p);
  } catch (...) {
  }
  delete p;
}

dda_status dda_profile_enable(dda_problem *p, int on) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    HIPCHK(hipStreamSynchronize(p->st));
    p->prof.collect();
    p->prof.reset();
    p->prof.on = on != 0;
    return DDA_OK;
  });
}

dda_status dda_profile_only(dda_problem *p, const char *name) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    HIPCHK(hipStreamSynchronize(p->st));
    p->prof.collect();
    p->prof.only = name ? name : "";
    return DDA_OK;
  });
}

int dda_profile_count(dda_problem *p) { return p ? (int)p->prof.kinds.size() : 0; }

dda_status dda_profile_get(dda_problem *p, int idx, const char **name, long long *launches,
                           double *total_ms, double *bytes_per_launch) {
  return guarded([&]() -> dda_status {
    REQUIRE(p, DDA_EINVAL, "problem is NULL");
    HIPCHK(hipStreamSynchronize(p->st));
    p->prof.collect();
    REQUIRE(idx >= 0 && idx < (int)p->prof.kinds.size(), DDA_EINVAL, "profile index out of range");
    const auto &k = p->prof.kinds[idx];
    if (name) *name = k.name.c_str();
    long long n = 0;
    double ms = 0.0, bytes = 0.0;
    k.working(n, ms, bytes);
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    if (bytes_per_launch) *bytes_per_launch = n ? bytes / n : 0.0;
    return DDA_OK;
  });
}

}  // extern "C"
