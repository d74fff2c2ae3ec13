// Instantiations and launcher of the register z pass.
#include "fft_kernels.h"
#include "zpass_mr.h"

namespace dda {

// The compile-time roots against closed forms: cos(pi/3), sin(pi/6), cos(2pi/5) = (sqrt5-1)/4,
// sin(pi/4), cos(6pi/7), sin(5pi/7) = sin(2pi/7)
constexpr bool cx_near(double a, double b) { return a - b < 2e-16 && b - a < 2e-16; }
static_assert(cx_near(cx_cos2pi(1, 6), 0.5) && cx_near(cx_sin2pi(1, 12), 0.5), "roots");
static_assert(cx_near(cx_cos2pi(1, 5), 0.30901699437494742410), "roots");
static_assert(cx_near(cx_sin2pi(1, 8), 0.70710678118654752440), "roots");
static_assert(cx_near(cx_cos2pi(3, 7), -0.90096886790241912624), "roots");
static_assert(cx_near(cx_sin2pi(5, 14), 0.78183148246802980871), "roots");
static_assert(cx_cos2pi(5, 20) == 0.0 && cx_sin2pi(-3, 12) == -1.0, "roots");

namespace {
// Supported lengths n = G P: G, P even and at most 16 (registers per thread), with P = 2 G
// where that factorisation exists (no idle threads), else P <= G with G as small as the
// factorisation allows.  Other lengths use the LDS-staged z pass.
struct Split {
  int n, G, P;
};
constexpr Split kSplits[] = {
    {24, 6, 4},    {32, 4, 8},    {36, 6, 6},    {40, 10, 4},   {48, 8, 6},
    {56, 14, 4},   {60, 10, 6},   {64, 8, 8},    {72, 6, 12},   {80, 10, 8},
    {84, 14, 6},   {96, 12, 8},   {100, 10, 10}, {112, 14, 8},  {120, 12, 10},
    {128, 8, 16},  {140, 14, 10}, {144, 12, 12}, {160, 16, 10}, {168, 14, 12},
    {192, 16, 12}, {196, 14, 14}, {224, 16, 14}, {256, 16, 16},
};

template <typename T, int I = 0>
void launch_at(int n, unsigned grid, int threads, size_t lds, hipStream_t st, cplx<T> *data,
               const cplx<T> *tw, const cplx<T> *khat, const ZRArgs &a) {
  if constexpr (I < (int)(sizeof(kSplits) / sizeof(kSplits[0]))) {
    constexpr Split s = kSplits[I];
    if (n != s.n) {
      launch_at<T, I + 1>(n, grid, threads, lds, st, data, tw, khat, a);
      return;
    }
    auto fn = k_zpass_mr<T, s.G, s.P>;
    set_lds_limit((const void *)fn, lds);
    hipLaunchKernelGGL(fn, dim3(grid), dim3(threads), lds, st, data, tw, khat, a);
  } else {
    REQUIRE(false, DDA_EUNSUPPORTED, "mixed-radix z pass: length %d", n);
  }
}
}  // namespace

bool zmr_split(int n, int *G, int *P) {
  for (const Split &s : kSplits)
    if (s.n == n) {
      *G = s.G;
      *P = s.P;
      return true;
    }
  return false;
}

template <typename T>
void zmr_launch(int n, unsigned grid, int threads, size_t lds, hipStream_t st, cplx<T> *data,
                const cplx<T> *tw, const cplx<T> *khat, const ZRArgs &a) {
  launch_at<T>(n, grid, threads, lds, st, data, tw, khat, a);
}

template void zmr_launch<double>(int, unsigned, int, size_t, hipStream_t, double2 *,
                                 const double2 *, const double2 *, const ZRArgs &);
template void zmr_launch<float>(int, unsigned, int, size_t, hipStream_t, float2 *, const float2 *,
                                const float2 *, const ZRArgs &);

}  // namespace dda
