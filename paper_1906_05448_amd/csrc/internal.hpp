// internal.hpp - context layout and kernel launchers shared by the library's
// translation units. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "d3q19.hpp"
#include "lbm.h"

namespace lbm {

// Error bits latched on the device and reported by the next sync call.
enum : uint32_t { kErrUnstable = 1u, kErrOverlap = 2u, kErrCapacity = 4u };

// Lattice extent plus the launch geometry of the dense kernels. Blocks are
// 64 x 4 threads (one wavefront per 64-node x-run); the flat block id is
// remapped so that consecutive tiles land on the same XCD (the hardware deals
// workgroups round-robin over the 8 XCDs, each with its own L2).
struct Dims {
  int nx, ny, nz;
  uint32_t N;       // nodes
  uint32_t gx, gy;  // tiles along x (64 wide) and y (4 tall)
  uint32_t ntiles;  // gx * gy * nz
  uint32_t per_xcd; // ceil(ntiles / 8)
};

inline Dims make_dims(int nx, int ny, int nz) {
  Dims d;
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.N = (uint32_t)nx * (uint32_t)ny * (uint32_t)nz;
  d.gx = (uint32_t)(nx + 63) / 64;
  d.gy = (uint32_t)(ny + 3) / 4;
  d.ntiles = d.gx * d.gy * (uint32_t)nz;
  d.per_xcd = (d.ntiles + 7) / 8;
  return d;
}

// Optional per-kernel timing with HIP events on the context's stream.
struct Profiler {
  struct Pair {
    hipEvent_t a, b;
    int cls;
  };
  bool on = false;
  std::vector<Pair> pending;
  std::vector<hipEvent_t> pool;
  double ms[LBM_NPROF] = {};
  int64_t launches[LBM_NPROF] = {};

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  // Waits for every pending pair and folds it into the totals.
  hipError_t harvest() {
    hipError_t st = hipSuccess;
    for (auto& p : pending) {
      float t = 0.0f;
      hipError_t e = hipEventSynchronize(p.b);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, p.a, p.b);
      if (e != hipSuccess) st = e;
      ms[p.cls] += t;
      launches[p.cls] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    return st;
  }
  ~Profiler() {
    (void)harvest();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct Ctx {
  lbm_config cfg;
  hipStream_t stream;
  int device;
  Dims dims;
  MrtRates rates;
  float3 body_force;
  // Workspace slices (device pointers).
  void* f_cur;      // post-collision shifted populations, [19][N]
  void* f_nxt;
  uint32_t* err;    // latched error bits (one word)
  int64_t step;
  Profiler prof;
};

// Runs a launcher, bracketed by timing events when profiling is on.
template <class F>
hipError_t timed(Ctx& c, int cls, F&& launch) {
  if (!c.prof.on) return launch();
  hipEvent_t a = c.prof.take(), b = c.prof.take();
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, c.stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, c.stream);
  if (e != hipSuccess) return e;
  c.prof.pending.push_back({a, b, cls});
  if (c.prof.pending.size() > 8192) e = c.prof.harvest();
  return e;
}

// Dense kernels (dense.hip).
hipError_t launch_init_equilibrium(const Ctx& c, const float* u, const float* rho, void* f);
hipError_t launch_stream_collide(const Ctx& c, const void* A, void* B);
hipError_t launch_fields(const Ctx& c, const void* f, float* u, float* rho);

}  // namespace lbm

struct lbm_ctx {
  lbm::Ctx c;
};
