// Kernel launches with optional per-dispatch timing.
//
// Every kernel of the library is launched through mr::launch.  When a context
// has timing enabled it installs a LaunchTimer for the calling thread; each
// launch then goes through hipExtLaunchKernel with a start/stop event pair that
// the runtime attaches to the kernel dispatch itself, so the measured interval
// is the kernel's own execution and not the host's submission gaps.  Without a
// timer the launch is a plain hipLaunchKernel (also valid under stream capture).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <tuple>
#include <utility>
#include <vector>

namespace mr {

struct TimedLaunch {
  int family;
  hipEvent_t start, stop;
};

struct LaunchTimer {
  int family = 0;
  std::vector<TimedLaunch> *out = nullptr;
};

// The timer of the calling thread (nullptr: no timing).
extern thread_local LaunchTimer *tl_launch_timer;

template <typename... P, typename... A>
hipError_t launch(void (*kernel)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t s,
                  A... a) {
  static_assert(sizeof...(P) == sizeof...(A) && sizeof...(P) > 0, "kernel argument count");
  std::tuple<P...> args{static_cast<P>(a)...};
  LaunchTimer *t = tl_launch_timer;
  return std::apply(
      [&](auto &...x) -> hipError_t {
        void *ptrs[] = {static_cast<void *>(&x)...};
        if (!t || !t->out)
          return hipLaunchKernel(reinterpret_cast<const void *>(kernel), grid, block, ptrs, lds, s);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipError_t e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        if (e != hipSuccess) return e;
        e = hipExtLaunchKernel(reinterpret_cast<const void *>(kernel), grid, block, ptrs, lds, s,
                               e0, e1, 0);
        t->out->push_back({t->family, e0, e1});
        return e;
      },
      args);
}

}  // namespace mr
