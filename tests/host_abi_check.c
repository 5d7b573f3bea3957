/* Host-side checks of the C ABI that need no GPU: configuration validation
 * and workspace planning over valid and invalid configurations (the sphere
 * support and link capacity bounds, pipe-wall marker and link counts, size
 * limits), and the argument checks of every entry point given null
 * handles or pointers. Built with the address and undefined-behaviour
 * sanitizers on the host code by tests/test_host_sanitizers.py; prints one
 * line per case (name, status, bytes) for the test to compare. */
#include <stdio.h>
#include <string.h>

#include "lbm.h"

static void size_case(const char* name, const lbm_config* c) {
  size_t b = 0;
  const int st = lbm_workspace_size(c, &b);
  printf("%s %d %zu\n", name, st, st == LBM_OK ? b : (size_t)0);
}

int main(void) {
  lbm_config c, d;
  lbm_config_default(&d);

  c = d;
  size_case("default", &c);
  c = d; c.nx = 512; c.ny = 512; c.nz = 512; c.store = LBM_STORE_F16S;
  size_case("dense512_f16", &c);
  c = d; c.nx = 1024; c.ny = 1024; c.nz = 1024; c.store = LBM_STORE_F32;
  size_case("dense1024_f32", &c);
  c = d; c.nx = 2048; c.ny = 1024; c.nz = 1024; c.store = LBM_STORE_F16S;
  size_case("too_many_nodes", &c);
  c = d; c.nx = 1024; c.ny = 1024; c.nz = 1025; c.store = LBM_STORE_F32;
  size_case("f32_offset_limit", &c);
  c = d; c.nx = 3;
  size_case("too_small", &c);
  c = d; c.tau = 0.5;
  size_case("tau_half", &c);
  c = d; c.s_q = 2.0;
  size_case("rate_two", &c);
  c = d; c.body_force[1] = 1.0 / 0.0;
  size_case("force_inf", &c);
  c = d; c.store = 7;
  size_case("bad_store", &c);
  c = d; c.bc = 9;
  size_case("bad_bc", &c);
  c = d; c.lattice = 5;
  size_case("bad_lattice", &c);

  /* particles */
  c = d; c.nx = 128; c.ny = 128; c.nz = 128; c.bc = LBM_BC_IBB; c.max_particles = 98; c.max_radius = 8.0;
  size_case("ibb_128_98", &c);
  c.ibb_max_order = 1;
  size_case("ibb_linear", &c);
  c.ibb_max_order = 3;
  size_case("ibb_order3", &c);
  c = d; c.nx = 128; c.ny = 128; c.nz = 128; c.bc = LBM_BC_IBM; c.ibm_retraction = 0.4; c.max_particles = 98;
  c.max_radius = 8.0;
  size_case("ibm_128_98", &c);
  c.ibm_retraction = 0.0;
  size_case("ibm_rd0", &c);
  c.ibm_retraction = 2.5;
  size_case("ibm_rd_large", &c);
  c.ibm_retraction = 0.4; c.max_radius = 13.0;
  size_case("ibm_box_too_wide", &c);
  c.max_radius = 8.0; c.ibm_iters = 17;
  size_case("ibm_iters", &c);
  c = d; c.nx = 512; c.ny = 512; c.nz = 512; c.bc = LBM_BC_IBB; c.store = LBM_STORE_F16S; c.max_particles = 6250;
  c.max_radius = 8.0;
  size_case("ibb_512_6250", &c);
  c.bc = LBM_BC_IBM; c.ibm_retraction = 0.4;
  size_case("ibm_512_6250", &c);
  c = d; c.nx = 40; c.ny = 40; c.nz = 40; c.bc = LBM_BC_IBB; c.max_particles = 2; c.max_radius = 20.0;
  size_case("radius_box", &c);
  c = d; c.bc = LBM_BC_NONE; c.max_particles = 4; c.max_radius = 4.0;
  size_case("particles_no_bc", &c);
  c = d; c.bc = LBM_BC_IBB; c.max_particles = 4; c.max_radius = 4.0; c.coll_restitution = 1.5;
  size_case("restitution", &c);

  /* pipe walls */
  c = d; c.nx = 160; c.ny = 160; c.nz = 480; c.bc = LBM_BC_IBB; c.ibb_max_order = 1; c.wall = LBM_WALL_PIPE_Z;
  c.pipe_radius = 74.5; c.pipe_cx = 79.5; c.pipe_cy = 79.5;
  size_case("pipe_ibb", &c);
  c.lattice = LBM_LATTICE_D3Q27;
  size_case("pipe_d3q27", &c);
  c.tau_bulk = 0.8;
  size_case("pipe_d3q27_bulk", &c);
  c.tau_bulk = 0.3;
  size_case("pipe_d3q27_bad_bulk", &c);
  c.tau_bulk = 0.0; c.store = LBM_STORE_F16S;
  size_case("pipe_d3q27_f16", &c);
  c = d; c.nx = 160; c.ny = 160; c.nz = 48; c.bc = LBM_BC_IBM; c.ibm_retraction = 0.4; c.wall = LBM_WALL_PIPE_Z;
  c.pipe_radius = 74.5; c.pipe_cx = 79.5; c.pipe_cy = 79.5;
  size_case("pipe_ibm", &c);
  c.pipe_radius = 0.5;
  size_case("pipe_radius_small", &c);
  c = d; c.wall = LBM_WALL_PIPE_Z; c.pipe_radius = 10.0; c.pipe_cx = 16.0; c.pipe_cy = 16.0;
  size_case("pipe_no_bc", &c);
  c = d; c.tau_bulk = 0.7;
  size_case("d3q19_bulk", &c);

  /* null arguments */
  size_t b = 0;
  printf("size_null_cfg %d\n", lbm_workspace_size(NULL, &b));
  printf("size_null_out %d\n", lbm_workspace_size(&d, NULL));
  lbm_ctx* ctx = NULL;
  printf("init_null_cfg %d\n", lbm_init(NULL, NULL, 0, NULL, &ctx));
  printf("init_null_out %d\n", lbm_init(&d, NULL, 0, NULL, NULL));
  printf("step_null %d\n", lbm_step(NULL, 1));
  printf("sync_null %d\n", lbm_sync(NULL));
  int64_t s64 = 0;
  printf("count_null %d\n", lbm_step_count(NULL, &s64));
  printf("state_size_null %d\n", lbm_state_size(NULL, &b));
  printf("get_state_null %d\n", lbm_get_state(NULL, NULL, 0));
  printf("set_state_null %d\n", lbm_set_state(NULL, NULL, 0));
  printf("set_fields_null %d\n", lbm_set_fields(NULL, NULL, NULL));
  printf("get_fields_null %d\n", lbm_get_fields(NULL, NULL, NULL));
  printf("set_particles_null %d\n", lbm_set_particles(NULL, 0, NULL, NULL, NULL, NULL, NULL, 0, 0));
  int32_t np = 0;
  printf("particle_count_null %d\n", lbm_particle_count(NULL, &np));
  printf("forces_null %d\n", lbm_forces(NULL, NULL, NULL, NULL));
  printf("link_count_null %d\n", lbm_link_count(NULL, &s64));
  printf("geometry_null %d\n", lbm_geometry_counts(NULL, &s64, &s64));
  printf("support_null %d\n", lbm_ibm_support(NULL, &s64, &s64));
  lbm_stats_t st;
  memset(&st, 0, sizeof(st));
  printf("stats_null %d\n", lbm_stats(NULL, 0, 0.25, &st, NULL));
  printf("spectrum_null %d\n", lbm_spectrum(NULL, 1, 8, NULL, NULL));
  printf("budget_null %d\n", lbm_pipe_budget_add(NULL));
  printf("profile_null %d\n", lbm_profile_enable(NULL, 1));
  printf("overlap_null %d\n", lbm_set_overlap(NULL, 1));
  printf("corrector_set_null %d\n", lbm_corrector_set(NULL, NULL, 0.0, 10.0, 0.03));
  printf("mlp_size %zu\n", lbm_mlp_workspace_size());
  printf("mlp_init_null %d\n", lbm_mlp_init(NULL, 0, NULL, NULL, NULL));
  printf("mlp_forward_null %d\n", lbm_mlp_forward(NULL, NULL, 1, NULL));
  printf("mlp_noalloc_null %d\n", lbm_mlp_gradient_noalloc(NULL, NULL, NULL, 1, NULL, NULL, NULL));
  printf("mlp_noalloc_n0 %d\n", lbm_mlp_gradient_noalloc(NULL, NULL, NULL, 0, NULL, NULL, NULL));
  lbm_destroy(NULL);
  lbm_mlp_destroy(NULL);
  for (int code = -8; code <= 2; ++code) {
    const char* t = lbm_strerror(code);
    printf("strerror %d %s\n", code, t ? "text" : "null");
  }
  return 0;
}
