// Context baselines for the CPU figures beside the oracle: the C++ standard library's sorts on one
// thread, timed inside the call.  TEST INFRASTRUCTURE ONLY (the benchmark's CPU-baseline leg).
#include <algorithm>
#include <chrono>
#include <cstddef>

namespace {
template <class F>
double seconds(F&& f) {
    const auto t0 = std::chrono::steady_clock::now();
    f();
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}
}  // namespace

extern "C" {
// Sorts a[0, n) ascending with std::sort; returns the seconds it took.
double ctx_std_sort_f64(double* a, size_t n) { return seconds([&] { std::sort(a, a + n); }); }
// Sorts a[0, n) ascending with std::stable_sort; returns the seconds it took.
double ctx_std_stable_sort_f64(double* a, size_t n) { return seconds([&] { std::stable_sort(a, a + n); }); }
}
