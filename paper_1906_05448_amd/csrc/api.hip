// api.hip - the extern "C" boundary: configuration checks, workspace
// carving, and the host-side sequencing of the kernels on the caller's
// stream. No kernel arithmetic lives here.
#include <math.h>
#include <new>
#include <string.h>

#include "internal.hpp"

using namespace lbm;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) & ~(kAlign - 1); }

size_t pop_bytes(const lbm_config& c) {
  const size_t N = (size_t)c.nx * (size_t)c.ny * (size_t)c.nz;
  const size_t elem = c.store == LBM_STORE_F32 ? 4 : 2;
  return align_up((size_t)kQ * N * elem);
}

// Workspace plan: offsets of every slice for a configuration.
struct Plan {
  size_t f_a, f_b, err, total;
};

Plan plan(const lbm_config& c) {
  Plan p;
  size_t off = 0;
  p.f_a = off;
  off += pop_bytes(c);
  p.f_b = off;
  off += pop_bytes(c);
  p.err = off;
  off += kAlign;
  p.total = off;
  return p;
}

bool rate_ok(double s) { return s > 0.0 && s < 2.0; }

int check_config(const lbm_config* c) {
  if (!c) return LBM_E_ARG;
  if (c->nx < 4 || c->ny < 4 || c->nz < 4) return LBM_E_ARG;
  const double N = (double)c->nx * (double)c->ny * (double)c->nz;
  if (N > 2147483647.0) return LBM_E_SIZE;
  if (!(c->tau > 0.5) || !isfinite(c->tau)) return LBM_E_ARG;
  if (!rate_ok(c->s_e) || !rate_ok(c->s_eps) || !rate_ok(c->s_q) || !rate_ok(c->s_pi) || !rate_ok(c->s_m))
    return LBM_E_ARG;
  for (int k = 0; k < 3; ++k)
    if (!isfinite(c->body_force[k])) return LBM_E_ARG;
  if (c->store != LBM_STORE_F32 && c->store != LBM_STORE_F16S) return LBM_E_ARG;
  if (c->bc != LBM_BC_NONE) return LBM_E_ARG;  // particle treatments not in this build yet
  if (c->wall != LBM_WALL_NONE) return LBM_E_ARG;
  return LBM_OK;
}

int hip_status(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_E_HIP; }

// Reads and clears the latched device error word (waits for the stream).
int drain_errors(Ctx& c) {
  uint32_t bits = 0;
  if (hipMemcpyAsync(&bits, c.err, sizeof(bits), hipMemcpyDeviceToHost, c.stream) != hipSuccess) return LBM_E_HIP;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return LBM_E_HIP;
  if (bits) {
    if (hipMemsetAsync(c.err, 0, sizeof(uint32_t), c.stream) != hipSuccess) return LBM_E_HIP;
    if (bits & kErrUnstable) return LBM_E_UNSTABLE;
    if (bits & kErrOverlap) return LBM_E_OVERLAP;
    if (bits & kErrCapacity) return LBM_E_SIZE;
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

void lbm_config_default(lbm_config* cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->nx = cfg->ny = cfg->nz = 32;
  cfg->tau = 0.6;
  cfg->s_e = 1.19;
  cfg->s_eps = 1.4;
  cfg->s_q = 1.2;
  cfg->s_pi = 1.4;
  cfg->s_m = 1.98;
  cfg->bc = LBM_BC_NONE;
  cfg->ibb_max_order = 2;
  cfg->ibm_retraction = 0.0;
  cfg->ibm_iters = 2;
  cfg->store = LBM_STORE_F32;
  cfg->wall = LBM_WALL_NONE;
  cfg->coll_restitution = 0.97;
  cfg->coll_tc_steps = 8.0;
}

int lbm_workspace_size(const lbm_config* cfg, size_t* bytes) {
  const int st = check_config(cfg);
  if (st != LBM_OK) return st;
  if (!bytes) return LBM_E_ARG;
  *bytes = plan(*cfg).total;
  return LBM_OK;
}

int lbm_init(const lbm_config* cfg, void* workspace, size_t bytes, void* stream, lbm_ctx** out) {
  if (!out) return LBM_E_ARG;
  *out = nullptr;
  const int st = check_config(cfg);
  if (st != LBM_OK) return st;
  if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return LBM_E_ARG;
  const Plan p = plan(*cfg);
  if (bytes < p.total) return LBM_E_SIZE;

  lbm_ctx* h = new (std::nothrow) lbm_ctx();
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  c.cfg = *cfg;
  c.stream = (hipStream_t)stream;
  if (hipGetDevice(&c.device) != hipSuccess) {
    delete h;
    return LBM_E_HIP;
  }
  c.dims = make_dims(cfg->nx, cfg->ny, cfg->nz);
  c.rates.s_nu = (float)(1.0 / cfg->tau);
  c.rates.s_e = (float)cfg->s_e;
  c.rates.s_eps = (float)cfg->s_eps;
  c.rates.s_q = (float)cfg->s_q;
  c.rates.s_pi = (float)cfg->s_pi;
  c.rates.s_m = (float)cfg->s_m;
  c.body_force = make_float3((float)cfg->body_force[0], (float)cfg->body_force[1], (float)cfg->body_force[2]);
  char* base = (char*)workspace;
  c.f_cur = base + p.f_a;
  c.f_nxt = base + p.f_b;
  c.err = (uint32_t*)(base + p.err);
  c.step = 0;

  // Start at rest, density 1: shifted populations are all zero.
  hipError_t e = hipMemsetAsync(c.f_cur, 0, pop_bytes(*cfg), c.stream);
  if (e == hipSuccess) e = hipMemsetAsync(c.err, 0, sizeof(uint32_t), c.stream);
  if (e != hipSuccess) {
    delete h;
    return LBM_E_HIP;
  }
  *out = h;
  return LBM_OK;
}

int lbm_set_fields_device(lbm_ctx* h, const float* u_dev, const float* rho_dev) {
  if (!h || !u_dev) return LBM_E_ARG;
  Ctx& c = h->c;
  c.step = 0;
  return hip_status(launch_init_equilibrium(c, u_dev, rho_dev, c.f_cur));
}

int lbm_set_fields(lbm_ctx* h, const float* u, const float* rho) {
  if (!h || !u) return LBM_E_ARG;
  Ctx& c = h->c;
  // Stage through the idle population buffer: it holds no state between
  // steps and is at least 16 bytes per node.
  const size_t N = c.dims.N;
  float* su = (float*)c.f_nxt;
  float* sr = rho ? su + 3 * N : nullptr;
  if (hipMemcpyAsync(su, u, 3 * N * sizeof(float), hipMemcpyHostToDevice, c.stream) != hipSuccess) return LBM_E_HIP;
  if (rho && hipMemcpyAsync(sr, rho, N * sizeof(float), hipMemcpyHostToDevice, c.stream) != hipSuccess)
    return LBM_E_HIP;
  int st = lbm_set_fields_device(h, su, sr);
  if (st != LBM_OK) return st;
  if (hipStreamSynchronize(c.stream) != hipSuccess) return LBM_E_HIP;
  return LBM_OK;
}

int lbm_step(lbm_ctx* h, int32_t nsteps) {
  if (!h || nsteps < 0) return LBM_E_ARG;
  Ctx& c = h->c;
  for (int32_t s = 0; s < nsteps; ++s) {
    hipError_t e = timed(c, LBM_K_STREAM_COLLIDE, [&] { return launch_stream_collide(c, c.f_cur, c.f_nxt); });
    if (e != hipSuccess) return LBM_E_HIP;
    void* t = c.f_cur;
    c.f_cur = c.f_nxt;
    c.f_nxt = t;
    ++c.step;
  }
  return LBM_OK;
}

int lbm_get_fields_device(lbm_ctx* h, float* u_dev, float* rho_dev) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  return hip_status(launch_fields(c, c.f_cur, u_dev, rho_dev));
}

int lbm_get_fields(lbm_ctx* h, float* u, float* rho) {
  if (!h) return LBM_E_ARG;
  Ctx& c = h->c;
  const size_t N = c.dims.N;
  float* su = (float*)c.f_nxt;
  float* sr = su + 3 * N;
  int st = lbm_get_fields_device(h, u ? su : nullptr, rho ? sr : nullptr);
  if (st != LBM_OK) return st;
  if (u && hipMemcpyAsync(u, su, 3 * N * sizeof(float), hipMemcpyDeviceToHost, c.stream) != hipSuccess)
    return LBM_E_HIP;
  if (rho && hipMemcpyAsync(rho, sr, N * sizeof(float), hipMemcpyDeviceToHost, c.stream) != hipSuccess)
    return LBM_E_HIP;
  return drain_errors(c);
}

int lbm_sync(lbm_ctx* h) {
  if (!h) return LBM_E_ARG;
  return drain_errors(h->c);
}

int lbm_step_count(const lbm_ctx* h, int64_t* step) {
  if (!h || !step) return LBM_E_ARG;
  *step = h->c.step;
  return LBM_OK;
}

int lbm_profile_enable(lbm_ctx* h, int32_t on) {
  if (!h) return LBM_E_ARG;
  h->c.prof.on = on != 0;
  return LBM_OK;
}

int lbm_profile_read(lbm_ctx* h, double* ms, int64_t* launches) {
  if (!h) return LBM_E_ARG;
  Profiler& p = h->c.prof;
  if (p.harvest() != hipSuccess) return LBM_E_HIP;
  for (int k = 0; k < LBM_NPROF; ++k) {
    if (ms) ms[k] = p.ms[k];
    if (launches) launches[k] = p.launches[k];
    p.ms[k] = 0.0;
    p.launches[k] = 0;
  }
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->c.stream);
  delete h;
}

const char* lbm_strerror(int status) {
  switch (status) {
    case LBM_OK: return "ok";
    case LBM_E_ARG: return "invalid argument or configuration";
    case LBM_E_HIP: return "HIP runtime call failed";
    case LBM_E_SIZE: return "workspace too small or capacity exceeded";
    case LBM_E_STATE: return "call not valid in the current state";
    case LBM_E_UNSTABLE: return "numerical instability: non-finite or |u| > 0.35";
    case LBM_E_OVERLAP: return "particles overlap by more than half a radius";
    default: return "unknown status";
  }
}

}  // extern "C"
