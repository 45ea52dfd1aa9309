// Host-side checks of the C ABI (include/clb.h) that need no GPU: parameter
// validation, derived constants, workspace sizes of every form, and the
// documented error codes for invalid and null arguments.  Built and run with
// AddressSanitizer and UndefinedBehaviorSanitizer by test_host_sanitizers.py
// (the library's host code instrumented, its device code not); every call
// here returns before any device work.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "clb3d.h"

#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #cond);      \
      return 1;                                                        \
    }                                                                  \
  } while (0)

static clb_params channel(int nx, int ny, double kn) {
  clb_params p;
  clb_params_default(&p);
  p.nx = nx;
  p.ny = ny;
  p.kn = kn;
  p.gx = 1e-6;
  return p;
}

static clb_params pressure(int nx, int ny, double kn) {
  clb_params p;
  clb_params_default(&p);
  p.nx = nx;
  p.ny = ny;
  p.kn = kn;
  p.xbc = CLB_X_PRESSURE;
  p.init = CLB_INIT_LINEAR_RHO;
  p.p_ratio = 1.8;
  return p;
}

int main() {
  // single channel: derivation, sizes, every invalid field
  clb_params p = channel(100, 20, 0.1);
  clb_derived d;
  EXPECT(clb_derive(&p, &d) == CLB_OK);
  EXPECT(d.s_nu > 0 && d.s_nu < 2 && d.s_q > 0 && d.s_q < 2 && d.r > 0 && d.r < 1);
  size_t n = 0;
  EXPECT(clb_workspace_size(&p, &n) == CLB_OK && n >= 2 * 72 * 128 * 20);
  struct Bad {
    const char* field;
    void (*set)(clb_params*);
  } bad[] = {
      {"nx", [](clb_params* q) { q->nx = 0; }},
      {"ny", [](clb_params* q) { q->ny = -3; }},
      {"xbc", [](clb_params* q) { q->xbc = 7; }},
      {"kn", [](clb_params* q) { q->kn = -1.0; }},
      {"kn", [](clb_params* q) { q->kn = NAN; }},
      {"a", [](clb_params* q) { q->a = -0.5; }},
      {"sigma", [](clb_params* q) { q->sigma = 2.5; }},
      {"A1", [](clb_params* q) { q->A1 = -1.0; }},
      {"A2", [](clb_params* q) { q->A2 = INFINITY; }},
      {"r", [](clb_params* q) { q->r = 1.5; }},
      {"s3", [](clb_params* q) { q->s3 = 2.0; }},
      {"s8", [](clb_params* q) { q->s8 = 0.0; }},
      {"gx/gy", [](clb_params* q) { q->gx = NAN; }},
      {"init", [](clb_params* q) { q->init = 9; }},
      {"tq_den", [](clb_params* q) { q->tq_den = 0.0; }},
      {"cbbsr_shift", [](clb_params* q) { q->cbbsr_shift = 3; }},
      {"forcing", [](clb_params* q) { q->forcing = 2; }},
  };
  for (const Bad& b : bad) {
    clb_params q = p;
    b.set(&q);
    EXPECT(clb_derive(&q, &d) == CLB_EINVAL);
    EXPECT(std::strncmp(clb_last_error(), b.field, std::strlen(b.field)) == 0);
    EXPECT(clb_workspace_size(&q, &n) == CLB_EINVAL);
  }
  clb_params q = pressure(100, 20, 0.1);
  q.gx = 1e-6;
  EXPECT(clb_derive(&q, &d) == CLB_EINVAL);   // no body force in pressure mode

  // null arguments of the single-channel entry points
  EXPECT(clb_derive(nullptr, &d) == CLB_EINVAL);
  EXPECT(clb_derive(&p, nullptr) == CLB_EINVAL);
  EXPECT(clb_workspace_size(&p, nullptr) == CLB_EINVAL);
  clb_ctx* c = nullptr;
  EXPECT(clb_init(&p, nullptr, 0, nullptr, &c) == CLB_EINVAL && c == nullptr);
  EXPECT(clb_init(&p, nullptr, 0, nullptr, nullptr) == CLB_EINVAL);
  int64_t steps = 0;
  int32_t ok = 0;
  double h = 0.0;
  EXPECT(clb_step(nullptr, 1) == CLB_EINVAL);
  EXPECT(clb_steps_done(nullptr, &steps) == CLB_EINVAL);
  EXPECT(clb_moments(nullptr, nullptr, nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb_column_sums(nullptr, nullptr, nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb_massflow(nullptr, nullptr, &h) == CLB_EINVAL);
  EXPECT(clb_flow_rate(nullptr, &h) == CLB_EINVAL);
  EXPECT(clb_pressure_deviation(nullptr, nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb_get_populations(nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb_set_populations(nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb_check_finite(nullptr, &ok) == CLB_EINVAL);
  EXPECT(clb_set_launch(nullptr, 1024, 1) == CLB_EINVAL);
  EXPECT(clb_set_steps_per_launch(nullptr, 2) == CLB_EINVAL);
  EXPECT(clb_set_pressure_path(nullptr, 0) == CLB_EINVAL);
  EXPECT(clb_set_graph_steps(nullptr, 8) == CLB_EINVAL);
  EXPECT(clb_set_check_every(nullptr, 8) == CLB_EINVAL);

  // 3-D duct step: validation and null handles
  clb3_params q3;
  clb3_params_default(&q3);
  q3.nx = 16;
  q3.ny = 12;
  q3.nz = 10;
  EXPECT(clb3_derive(&q3, &d) == CLB_OK && d.s_nu > 0 && d.s_nu < 2);
  EXPECT(clb3_workspace_size(&q3, &n) == CLB_OK && n >= 2 * 216 * 16 * 12 * 10);
  {
    clb3_params b3 = q3;
    b3.nz = 0;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3 = q3;
    b3.cbbsr_shift = 0;   // same-node specular source with walls in z
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3.zbc = CLB3_Z_PERIODIC;
    EXPECT(clb3_derive(&b3, &d) == CLB_OK);
    b3 = q3;
    b3.init = CLB_INIT_LINEAR_RHO;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3 = q3;
    b3.s_b = 2.0;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3 = q3;
    b3.kn = -1.0;
    EXPECT(clb3_workspace_size(&b3, &n) == CLB_EINVAL);
    // pressure-driven ducts: the ghost planes add 2 * 27 doubles per row of the cross-section
    size_t n_force = 0, n_press = 0;
    EXPECT(clb3_workspace_size(&q3, &n_force) == CLB_OK);
    b3 = q3;
    b3.xbc = CLB_X_PRESSURE;
    EXPECT(clb3_derive(&b3, &d) == CLB_OK);
    EXPECT(clb3_workspace_size(&b3, &n_press) == CLB_OK && n_press >= n_force + 2 * 27 * 8 * 12 * 10);
    b3.init = CLB_INIT_LINEAR_RHO;
    EXPECT(clb3_derive(&b3, &d) == CLB_OK);
    b3.nx = 1;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3.nx = 2;
    EXPECT(clb3_derive(&b3, &d) == CLB_OK);
    b3.gx = 1e-5;   // no body force in a pressure-driven duct
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3.gx = 0.0;
    b3.gz = 1e-5;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3.gz = 0.0;
    b3.p_ratio = 0.0;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3.p_ratio = NAN;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
    b3.p_ratio = 2.0;
    b3.rho_out = -1.0;
    EXPECT(clb3_workspace_size(&b3, &n) == CLB_EINVAL);
    b3.rho_out = 1.0;
    b3.xbc = 7;
    EXPECT(clb3_derive(&b3, &d) == CLB_EINVAL);
  }
  EXPECT(clb3_derive(nullptr, &d) == CLB_EINVAL);
  EXPECT(clb3_derive(&q3, nullptr) == CLB_EINVAL);
  EXPECT(clb3_step(nullptr, 1) == CLB_EINVAL);
  EXPECT(clb3_flow_rate(nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb3_massflow(nullptr, nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb3_set_graph_steps(nullptr, 4) == CLB_EINVAL);
  EXPECT(clb3_pressure_deviation(nullptr, nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb3_destroy(nullptr) == CLB_EINVAL);
  clb3_ctx* c3 = nullptr;
  EXPECT(clb3_init(&q3, nullptr, n, nullptr, &c3) == CLB_EINVAL && c3 == nullptr);
  EXPECT(clb_destroy(nullptr) == CLB_EINVAL);

  // Kn-sweep batch
  clb_params ps[3] = {channel(4, 16, 0.1), channel(4, 32, 1.0), channel(7, 9, 3.0)};
  EXPECT(clb_batch_workspace_size(3, ps, &n) == CLB_OK && n >= 72 * (64 + 128 + 63));
  EXPECT(clb_batch_workspace_size(0, ps, &n) == CLB_EINVAL);
  EXPECT(clb_batch_workspace_size(3, nullptr, &n) == CLB_EINVAL);
  EXPECT(clb_batch_workspace_size(3, ps, nullptr) == CLB_EINVAL);
  clb_params ps_bad[2] = {channel(4, 16, 0.1), pressure(10, 8, 0.1)};
  EXPECT(clb_batch_workspace_size(2, ps_bad, &n) == CLB_EINVAL);
  clb_batch* b = nullptr;
  EXPECT(clb_batch_init(3, ps, nullptr, 0, nullptr, &b) == CLB_EINVAL && b == nullptr);
  EXPECT(clb_batch_run(nullptr, 10, 0, 0.0, nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb_batch_flow_rate(nullptr, &h) == CLB_EINVAL);
  EXPECT(clb_batch_check_finite(nullptr, &ok) == CLB_EINVAL);
  EXPECT(clb_batch_destroy(nullptr) == CLB_EINVAL);

  // pressure batch
  clb_params pp[3] = {pressure(300, 10, 0.05), pressure(300, 10, 0.5), pressure(300, 10, 2.0)};
  EXPECT(clb_pbatch_workspace_size(3, pp, &n) == CLB_OK && n >= 3 * 2 * 72 * 512 * 10);
  clb_params pp_bad[2] = {pressure(300, 10, 0.05), pressure(300, 11, 0.5)};
  EXPECT(clb_pbatch_workspace_size(2, pp_bad, &n) == CLB_EINVAL);
  EXPECT(std::strncmp(clb_last_error(), "nx/ny", 5) == 0);
  clb_pbatch* pb = nullptr;
  EXPECT(clb_pbatch_init(3, pp, nullptr, 0, nullptr, &pb) == CLB_EINVAL && pb == nullptr);
  EXPECT(clb_pbatch_step(nullptr, 1) == CLB_EINVAL);
  EXPECT(clb_pbatch_run(nullptr, 10, 0, 0.0, nullptr, nullptr) == CLB_EINVAL);
  EXPECT(clb_pbatch_massflow(nullptr, &h, &h) == CLB_EINVAL);
  EXPECT(clb_pbatch_check_finite(nullptr, &ok) == CLB_EINVAL);
  EXPECT(clb_pbatch_destroy(nullptr) == CLB_EINVAL);

  // adjoint
  clb_params pa = pressure(200, 10, 0.1);
  EXPECT(clb_adjoint_workspace_size(&pa, 100, 10, &n) == CLB_OK && n > 0);
  EXPECT(clb_adjoint_workspace_size(&pa, 0, 1, &n) == CLB_EINVAL);
  EXPECT(clb_adjoint_workspace_size(&pa, 10, 11, &n) == CLB_EINVAL);
  EXPECT(clb_adjoint_workspace_size(&p, 10, 2, &n) == CLB_EINVAL);   // periodic
  clb_adjoint* ad = nullptr;
  EXPECT(clb_adjoint_init(&pa, 10, 2, nullptr, 0, nullptr, &ad) == CLB_EINVAL && ad == nullptr);
  double g[4];
  EXPECT(clb_adjoint_backward(nullptr, g) == CLB_EINVAL);
  EXPECT(clb_adjoint_destroy(nullptr) == CLB_EINVAL);

  std::printf("host checks ok\n");
  return 0;
}
