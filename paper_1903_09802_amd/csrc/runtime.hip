// Runtime pieces: error reporting, FFT plans (radix factorisation + twiddle tables),
// per-kernel event profiling, and the plain (setup) FFT launchers.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "fft_kernels.h"

namespace dda {

static thread_local char g_err[1024] = "";

void set_error(const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

const char *get_error() { return g_err; }

// ----------------------------------------------------------------------------- plans

bool factor_7smooth(int n, FftPlan &plan) {
  plan.n = n;
  plan.nrad = 0;
  int m = n;
  auto push = [&](int r) {
    if (plan.nrad >= kMaxRadices) return false;
    plan.rad[plan.nrad++] = r;
    m /= r;
    return true;
  };
  while (m % 8 == 0) if (!push(8)) return false;
  while (m % 4 == 0) if (!push(4)) return false;
  while (m % 2 == 0) if (!push(2)) return false;
  while (m % 7 == 0) if (!push(7)) return false;
  while (m % 5 == 0) if (!push(5)) return false;
  while (m % 3 == 0) if (!push(3)) return false;
  return m == 1;
}

void plan_create(FftPlan &plan, int n) {
  REQUIRE(n >= 1 && n <= kMaxFft, DDA_EUNSUPPORTED, "FFT length %d outside [1, %d]", n, kMaxFft);
  REQUIRE(factor_7smooth(n, plan), DDA_EUNSUPPORTED,
          "FFT length %d has a prime factor above 7 (grid dimensions must be 7-smooth)", n);
  std::vector<double2> t64(n);
  std::vector<float2> t32(n);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int t = 0; t < n; ++t) {
    const long double ang = two_pi * (long double)t / (long double)n;
    const double c = (double)cosl(ang), s = -(double)sinl(ang);
    t64[t] = make_double2(c, s);
    t32[t] = make_float2((float)c, (float)s);
  }
  HIPCHK(hipMalloc(&plan.tw64, sizeof(double2) * n));
  HIPCHK(hipMalloc(&plan.tw32, sizeof(float2) * n));
  HIPCHK(hipMemcpy(plan.tw64, t64.data(), sizeof(double2) * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(plan.tw32, t32.data(), sizeof(float2) * n, hipMemcpyHostToDevice));
}

void plan_destroy(FftPlan &plan) {
  if (plan.tw64) (void)hipFree(plan.tw64);
  if (plan.tw32) (void)hipFree(plan.tw32);
  plan.tw64 = nullptr;
  plan.tw32 = nullptr;
}

// ----------------------------------------------------------------------------- profiling

int Profiler::kind_id(const char *name) {
  for (size_t i = 0; i < kinds.size(); ++i)
    if (kinds[i].name == name) return (int)i;
  Kind k;
  k.name = name;
  kinds.push_back(k);
  return (int)kinds.size() - 1;
}

hipEvent_t Profiler::get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

void Profiler::collect() {
  for (auto &pd : pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pd.a, pd.b) == hipSuccess) {
      kinds[pd.kind].ms.push_back(ms);
      kinds[pd.kind].bytes.push_back(pd.bytes);
    }
    pool.push_back(pd.a);
    pool.push_back(pd.b);
  }
  pending.clear();
}

void Profiler::Kind::working(long long &n, double &total_ms, double &total_bytes) const {
  float mx = 0.f;
  for (float v : ms) mx = v > mx ? v : mx;
  n = 0;
  total_ms = total_bytes = 0.0;
  for (size_t i = 0; i < ms.size(); ++i)
    if (ms[i] >= 0.02f * mx) {
      ++n;
      total_ms += ms[i];
      total_bytes += bytes[i];
    }
}

void Profiler::reset() {
  for (auto &k : kinds) {
    k.ms.clear();
    k.bytes.clear();
  }
}

void Profiler::destroy() {
  for (auto &pd : pending) {
    pool.push_back(pd.a);
    pool.push_back(pd.b);
  }
  pending.clear();
  for (auto e : pool) (void)hipEventDestroy(e);
  pool.clear();
}

KTimer::KTimer(Profiler *p, hipStream_t s, const char *name, double bytes) : prof(p), st(s) {
  if (!prof || !prof->on) {
    prof = nullptr;
    return;
  }
  if (!prof->only.empty() && prof->only != name) {
    prof = nullptr;
    return;
  }
  const int kind = prof->kind_id(name);
  a = prof->get_event();
  b = prof->get_event();
  HIPCHK(hipEventRecord(a, st));
  prof->pending.push_back(Profiler::Pending{kind, bytes, a, b});
}

KTimer::~KTimer() {
  if (prof) (void)hipEventRecord(b, st);
}

// ----------------------------------------------------------------------------- plain transforms

void fft_rows_plain(dda_problem *p, const FftPlan &pl, double2 *data, long long rows, int inverse) {
  RowArgs a{};
  a.rows = rows;
  a.n_in = pl.n;
  a.n_out = pl.n;
  a.in_stride = pl.n;
  a.out_stride = pl.n;
  a.sign = inverse ? 1 : -1;
  launch_rows<double, ROW_PLAIN, double2, double2>(p, pl, data, data, a, "fft_rows_setup",
                                                   32.0 * rows * pl.n);
}

void fft_strided_plain(dda_problem *p, const FftPlan &pl, double2 *data, long long batch,
                       long long width, int inverse) {
  launch_strided<double>(p, pl, data, data, batch, width, pl.n, pl.n, (long long)pl.n * width,
                         (long long)pl.n * width, inverse ? 1 : -1, "fft_strided_setup",
                         32.0 * batch * width * pl.n);
}

// ----------------------------------------------------------------------------- tile shapes

// Candidate shapes of a pass: rows per tile (x passes) halved from the LDS-bound maximum; along
// a strided axis (y passes) the maximum and half its columns, each with the launch rule's tiles
// per workgroup and with 2 and 8.
static std::vector<TileShape> tile_candidates(int max_tw, bool strided) {
  std::vector<TileShape> c;
  if (!strided) {
    for (int tw = max_tw; tw >= 1 && c.size() < 3; tw /= 2) c.push_back(TileShape{tw, 0});
    return c;
  }
  for (int tw : {max_tw, max_tw / 2}) {
    if (tw < 1) continue;
    for (int tpw : {0, 2, 8}) c.push_back(TileShape{tw, tpw});
  }
  return c;
}

static std::mutex g_tile_mu;
static std::map<std::tuple<int, int, int, int, int, int, int>, std::vector<TileShape>> g_tile;

void fft_tile_autotune(dda_problem *p, int first, int pi, int nrhs,
                       const std::function<void()> &apply) {
  if (const char *e = getenv("DDA_FFT_TUNE"))
    if (atoi(e) == 0) return;
  if (const char *f = getenv("DDA_FFT_FORCE")) {  // "rows,columns,tiles": every pass, for tests
    int rtw = 0, stw = 0, stpw = 0;
    REQUIRE(sscanf(f, "%d,%d,%d", &rtw, &stw, &stpw) == 3 && rtw >= 1 && stw >= 1 && stpw >= 1,
            DDA_EINVAL, "DDA_FFT_FORCE=\"%s\": want \"rows,columns,tiles\", each >= 1", f);
    for (int k = 0; k < 4; ++k)
      p->tile[first + k][pi] = (k == 1 || k == 2) ? TileShape{stw, stpw} : TileShape{rtw, 0};
    return;
  }
  const bool op = first == FP_OP_X_FWD;
  const auto key = std::make_tuple(p->dev, p->nx, p->ny, p->nz, nrhs, pi, first);
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    const auto it = g_tile.find(key);
    if (it != g_tile.end()) {
      for (int k = 0; k < 4; ++k) p->tile[first + k][pi] = it->second[k];
      return;
    }
  }
  const FftPlan *plans[4] = {op ? &p->px : &p->ux, op ? &p->py : &p->uy, op ? &p->py : &p->uy,
                             op ? &p->px : &p->ux};
  const char *stem[4] = {"x_fwd", "y_fwd", "y_inv", "x_inv"};
  std::vector<TileShape> cand[4];
  char name[4][32];
  size_t rounds = 0;
  for (int k = 0; k < 4; ++k) {
    const int n = plans[k]->n;
    const int max_tw = pi == 0 ? tile_cols<double>(n) : tile_cols<float>(n);
    cand[k] = tile_candidates(max_tw, k == 1 || k == 2);
    rounds = std::max(rounds, cand[k].size());
    snprintf(name[k], sizeof name[k], "%s_%s_%s", op ? "op" : "pc", stem[k], pi == 0 ? "f64" : "f32");
  }
  // time with a profiler of its own and every right-hand side live
  Profiler saved;
  std::swap(saved, p->prof);
  p->prof.on = true;
  const int *act = p->act;
  p->act = nullptr;
  p->tune_xy = 1;  // only the four timed passes run
  TileShape best[4];
  double best_ms[4] = {1e30, 1e30, 1e30, 1e30};
  try {
    for (int k = 0; k < 4; ++k) p->tile[first + k][pi] = TileShape{};
    apply();  // warm
    HIPCHK(hipStreamSynchronize(p->st));
    p->prof.collect();
    for (size_t c = 0; c < rounds; ++c) {
      for (int k = 0; k < 4; ++k) p->tile[first + k][pi] = cand[k][std::min(c, cand[k].size() - 1)];
      p->prof.reset();
      apply();
      HIPCHK(hipStreamSynchronize(p->st));
      p->prof.collect();
      for (int k = 0; k < 4; ++k) {
        if (c >= cand[k].size()) continue;
        for (const auto &kd : p->prof.kinds) {
          if (kd.name != name[k] || kd.ms.empty()) continue;
          double t = 0;
          for (float v : kd.ms) t += v;
          t /= kd.ms.size();
          // a shape other than the first must win by 3 %, so timing noise keeps the rule's
          if (t < best_ms[k] * (c == 0 ? 1.0 : 0.97)) {
            best_ms[k] = t;
            best[k] = cand[k][c];
          }
        }
      }
    }
  } catch (...) {
    p->prof.destroy();
    std::swap(saved, p->prof);
    p->act = act;
    p->tune_xy = 0;
    throw;
  }
  p->prof.destroy();
  std::swap(saved, p->prof);
  p->act = act;
  p->tune_xy = 0;
  std::vector<TileShape> chosen(4);
  for (int k = 0; k < 4; ++k) {
    // the first candidate is the launch rule's own shape: keep it as "rule" (zeros)
    chosen[k] = (best[k].tw == cand[k][0].tw && best[k].tpw == cand[k][0].tpw) ? TileShape{} : best[k];
    p->tile[first + k][pi] = chosen[k];
  }
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile[key] = chosen;
}

}  // namespace dda
