// Host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.
//
// This translation unit includes the library's API source, so its file-local
// helpers are reachable, and is compiled for the host only (no device code,
// no kernel is launched).  It drives what runs on the CPU:
//   * the size registry and cbs_axis_supported over every length up to 4200;
//   * the twiddle tables of every registered split, each written into a heap
//     buffer of exactly the axis length (an overrun is a heap-buffer-overflow),
//     against exp(-2 pi i j2 k1 / n) in FP64;
//   * the workspace carve-ups of a plan, a batch and the stretched layer: each
//     region 256-byte aligned, in order, large enough, no overflow at 1024^3;
//   * the argument checks of every entry point (null plan, bad grids, optics,
//     workspaces, options, sources, boxes, layer parameters), on a plan object
//     laid out on the host, all of which must fail before any device work;
//   * the source set-up of a valid call (plane wave at normal and oblique
//     incidence, point, field) and its wave vector;
//   * the half-maximum interpolation of the lens figures on profiles whose
//     width is known exactly;
//   * with no GPU present: plan creation and the allocation-free solve up to
//     their first HIP call, and the clean-up after its failure (the leak
//     checker sees anything left behind).
// Prints "host checks passed" and exits 0 when every check holds.

#include "../../paper_2506_15411_amd/csrc/cbs_api.hip"

#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <vector>

static int g_failed = 0;
static int g_checks = 0;

#define CHECK(cond)                                                                  \
  do {                                                                               \
    ++g_checks;                                                                      \
    if (!(cond)) {                                                                   \
      std::fprintf(stderr, "%s:%d: check failed: %s (last error: %s)\n", __FILE__,  \
                   __LINE__, #cond, cbs_last_error());                              \
      ++g_failed;                                                                    \
    }                                                                                \
  } while (0)

namespace {

using cbs::SizeOps;

std::vector<int> registry_checks() {
  std::vector<int> sizes;
  for (int n = -3; n <= 4200; ++n) {
    const SizeOps* o = cbs::find_size(n);
    const int sx = cbs_axis_supported(0, n), sy = cbs_axis_supported(1, n);
    const int sz = cbs_axis_supported(2, n);
    CHECK(sx == (o != nullptr) && sy == sx);
    CHECK(!cbs_axis_supported(-1, n) && !cbs_axis_supported(3, n));
    if (!o) {
      CHECK(!sz);
      continue;
    }
    sizes.push_back(n);
    CHECK(o->n == n && o->n1 * o->n2 == n && o->n1 >= 1 && o->n2 >= 1);
    CHECK(o->k1 != nullptr && o->ky != nullptr && o->k1_rows >= 1);
    CHECK(n <= kMaxAxis);
    CHECK(sz == (o->kz != nullptr));
    if (o->kz) CHECK(o->z1 * o->z2 == n && o->z1 >= 1 && o->z2 >= 1);
  }
  CHECK(sizes.size() >= 10);
  return sizes;
}

void twiddle_checks(const std::vector<int>& sizes) {
  for (int n : sizes) {
    const SizeOps* o = cbs::find_size(n);
    const int splits[2][2] = {{o->n1, o->n2}, {o->z1, o->z2}};
    for (int s = 0; s < (o->kz ? 2 : 1); ++s) {
      const int n1 = splits[s][0], n2 = splits[s][1];
      std::unique_ptr<float2[]> t(new float2[n]);
      fill_twiddles(t.get(), n1, n2);
      double worst = 0.0;
      for (int j2 = 0; j2 < n2; ++j2)
        for (int k1 = 0; k1 < n1; ++k1) {
          const double ang = -2.0 * M_PI * double(j2) * double(k1) / double(n);
          const float2 w = t[(size_t)j2 * n1 + k1];
          worst = std::max(worst, std::hypot(w.x - std::cos(ang), w.y - std::sin(ang)));
        }
      CHECK(worst < 1e-7);
    }
  }
}

void layout_checks(const std::vector<int>& sizes) {
  std::vector<std::array<int, 3>> grids = {{2, 2, 2}, {8, 8, 12}, {64, 64, 64},
                                           {275, 275, 315}, {621, 621, 261}, {25, 27, 15}};
  for (int n : sizes)
    if (cbs::find_size(n)->kz) grids.push_back({n, n, n});
  for (const auto& g : grids) {
    const int nx = g[0], ny = g[1], nz = g[2];
    if (!cbs_axis_supported(0, nx) || !cbs_axis_supported(1, ny) || !cbs_axis_supported(2, nz))
      continue;
    Layout L;
    CHECK(layout_of(nx, ny, nz, L));
    CHECK(cbs_plan_workspace_bytes(nx, ny, nz) == L.total);
    const size_t N = (size_t)nx * ny * nz;
    const size_t regions[] = {L.W, L.V0, L.twx, L.twy, L.twz, L.phase, L.phx, L.phy,
                              L.partials, L.setup, L.hist, L.metrics, L.state, L.total};
    const size_t need[] = {3 * (size_t)nz * ny * padded_pitch(nx) * sizeof(float2),
                           N * sizeof(float2), nx * sizeof(float2), ny * sizeof(float2),
                           nz * sizeof(float2), 3 * (size_t)nz * sizeof(float2),
                           nx * sizeof(float2), ny * sizeof(float2), 0, 0,
                           kHistCap * sizeof(double), 0, sizeof(DevState)};
    for (int r = 0; r + 1 < (int)(sizeof(regions) / sizeof(regions[0])); ++r) {
      CHECK(regions[r] % 256 == 0);
      CHECK(regions[r] + need[r] <= regions[r + 1]);
    }
    BatchLayout B;
    CHECK(!batch_layout(nx, ny, nz, 0, B) && !batch_layout(nx, ny, nz, kMaxIllum + 1, B));
    for (int c = 1; c <= kMaxIllum; ++c) {
      CHECK(batch_layout(nx, ny, nz, c, B));
      CHECK(B.W == 0 && B.partials >= (size_t)c * need[0]);
      CHECK(cbs_batch_workspace_bytes(nx, ny, nz, c) == B.total);
    }
    CHECK(cbs_batch_workspace_bytes(nx, ny, nz, 0) == 0);
    size_t prev = 0;
    for (int m = 0; m <= kScpmlMaxRestart + 1; ++m) {
      const size_t b = cbs_scpml_workspace_bytes(nx, ny, nz, m);
      if (m < 1 || m > kScpmlMaxRestart) {
        CHECK(b == 0);
        continue;
      }
      CHECK(b >= prev && b % 256 == 0);   // a basis field of a tiny grid is < 256 bytes
      CHECK(b >= (size_t)(m + 3) * 3 * N * sizeof(float2));
      prev = b;
    }
  }
  // unsupported or degenerate grids report no workspace
  CHECK(cbs_plan_workspace_bytes(1, 8, 8) == 0 && cbs_plan_workspace_bytes(8, 8, -4) == 0);
  CHECK(cbs_plan_workspace_bytes(37 * 41, 8, 8) == 0);
  CHECK(cbs_scpml_workspace_bytes(8, 8, 37 * 41, 4) == 0);
  // the largest registered cube: byte counts past 2^32 without overflow
  int big = 0;
  for (int n : sizes)
    if (cbs::find_size(n)->kz) big = std::max(big, n);
  const size_t wb = cbs_plan_workspace_bytes(big, big, big);
  CHECK(wb >= 4 * (size_t)big * big * big * sizeof(float2));
  CHECK(cbs_batch_workspace_bytes(big, big, big, kMaxIllum) >=
        (size_t)kMaxIllum * 3 * big * big * big * sizeof(float2));
}

// A plan laid out on the host (no HIP objects): argument checks only.
struct HostPlan {
  std::unique_ptr<unsigned char[]> mem;
  cbs_plan_s plan{};
  HostPlan(int nx, int ny, int nz, const int pml[3]) {
    const size_t bytes = cbs_plan_workspace_bytes(nx, ny, nz);
    mem.reset(new unsigned char[bytes + 256]);
    void* ws = mem.get() + (256 - reinterpret_cast<uintptr_t>(mem.get()) % 256) % 256;
    init_plan(&plan, nx, ny, nz, 1.064e-6 / 8, 1.064e-6, 1.0, pml, ws, nullptr);
  }
};

void argument_checks() {
  const int pml[3] = {2, 2, 3};
  const double lam = 1.064e-6, d = lam / 8;
  static unsigned char fake_dev[1];   // never dereferenced: every call below fails first
  void* dev = fake_dev;
  cbs_plan_t h = reinterpret_cast<cbs_plan_t>(0x1);

  // plan creation: arguments, grid, optics and workspace, before any HIP call
  CHECK(cbs_plan_create(nullptr, 8, 8, 12, d, lam, 1.0, pml, dev, 1 << 30, nullptr) ==
        CBS_E_INVALID);
  struct Bad {
    int nx, ny, nz;
    double pitch, lam, nbg;
    int pml[3];
  } bad[] = {{1, 8, 12, d, lam, 1, {0, 0, 0}},           {8, 8, 37 * 41, d, lam, 1, {0, 0, 0}},
             {8, 8, 12, 0, lam, 1, {0, 0, 0}},           {8, 8, 12, -d, lam, 1, {0, 0, 0}},
             {8, 8, 12, NAN, lam, 1, {0, 0, 0}},         {8, 8, 12, INFINITY, lam, 1, {0, 0, 0}},
             {8, 8, 12, d, 0, 1, {0, 0, 0}},             {8, 8, 12, d, NAN, 1, {0, 0, 0}},
             {8, 8, 12, d, lam, 0, {0, 0, 0}},           {8, 8, 12, d, lam, -1, {0, 0, 0}},
             {8, 8, 12, d, lam, INFINITY, {0, 0, 0}},    {8, 8, 12, d, lam, 1, {4, 0, 0}},
             {8, 8, 12, d, lam, 1, {0, 0, 6}},           {8, 8, 12, d, lam, 1, {-1, 0, 0}},
             {INT_MAX, 8, 12, d, lam, 1, {0, 0, 0}},     {8, INT_MIN, 12, d, lam, 1, {0, 0, 0}}};
  for (const Bad& b : bad) {
    h = reinterpret_cast<cbs_plan_t>(0x1);
    CHECK(cbs_plan_create(&h, b.nx, b.ny, b.nz, b.pitch, b.lam, b.nbg, b.pml, dev, 1 << 30,
                          nullptr) == CBS_E_INVALID);
    CHECK(h == nullptr && std::strlen(cbs_last_error()) > 0);
  }
  const size_t need = cbs_plan_workspace_bytes(8, 8, 12);
  alignas(256) static unsigned char aligned[512];
  CHECK(cbs_plan_create(&h, 8, 8, 12, d, lam, 1.0, pml, nullptr, need, nullptr) ==
        CBS_E_WORKSPACE);
  CHECK(cbs_plan_create(&h, 8, 8, 12, d, lam, 1.0, pml, aligned + 8, need, nullptr) ==
        CBS_E_WORKSPACE);
  CHECK(cbs_plan_create(&h, 8, 8, 12, d, lam, 1.0, pml, aligned, need - 1, nullptr) ==
        CBS_E_WORKSPACE);

  // every entry point on a null plan
  cbs_opts o{1e-4, 100, 10, 0};
  cbs_stats st{};
  cbs_source src{};
  const int lo[3] = {0, 0, 0}, hi[3] = {8, 8, 12};
  float ms[5];
  double hist[4];
  int done = 0, outstanding = 0;
  cbs_lens_figures fig{};
  cbs_scpml layer{0.75, 1, 8};
  CHECK(cbs_plan_set_pml_profile(nullptr, 2, 1.0) == CBS_E_INVALID);
  CHECK(cbs_plan_set_shift_factor(nullptr, 1.1) == CBS_E_INVALID);
  CHECK(cbs_set_permittivity(nullptr, dev, CBS_F32) == CBS_E_INVALID);
  CHECK(cbs_eps_shift(nullptr) == -1.0);
  CHECK(cbs_solve(nullptr, &src, dev, &o, &st) == CBS_E_INVALID);
  CHECK(cbs_adjoint_solve(nullptr, dev, &src, dev, &o, &st) == CBS_E_INVALID);
  CHECK(cbs_solve_begin(nullptr, 0, nullptr, &src, dev, &o) == CBS_E_INVALID);
  CHECK(cbs_solve_advance(nullptr, 1) == CBS_E_INVALID);
  CHECK(cbs_solve_poll(nullptr, &done, &outstanding) == CBS_E_INVALID);
  CHECK(cbs_solve_end(nullptr, &st) == CBS_E_INVALID);
  CHECK(cbs_solve_batch(nullptr, 1, &src, dev, &o, &st, dev, 1 << 30) == CBS_E_INVALID);
  CHECK(cbs_batch_step(nullptr, 1, 1, &done) == CBS_E_INVALID);
  CHECK(cbs_batch_step(nullptr, -1, 1, &done) == CBS_E_INVALID);
  CHECK(cbs_batch_step(nullptr, 0, 1, nullptr) == CBS_OK);   // nothing to step
  cbs_plan_t none[2] = {nullptr, nullptr};
  CHECK(cbs_batch_step(none, 2, 1, &done) == CBS_E_INVALID);
  CHECK(cbs_gradient(nullptr, dev, dev, lo, hi, 1.0, (float*)dev) == CBS_E_INVALID);
  CHECK(cbs_lens_metrics(nullptr, dev, lo, hi, 3.0, 1e-5, 1.0, &fig) == CBS_E_INVALID);
  CHECK(cbs_tfsf_source(nullptr, &src, lo, hi, dev) == CBS_E_INVALID);
  CHECK(cbs_apply_green(nullptr, dev, dev) == CBS_E_INVALID);
  CHECK(cbs_time_passes(nullptr, dev, 1, ms) == CBS_E_INVALID);
  CHECK(cbs_scpml_operator(nullptr, &layer, dev, dev, dev, 1 << 30) == CBS_E_INVALID);
  CHECK(cbs_solve_scpml(nullptr, &src, dev, &o, &layer, &st, dev, 1 << 30) == CBS_E_INVALID);
  CHECK(cbs_history(nullptr, hist, 4) == CBS_E_INVALID);
  CHECK(cbs_plan_destroy(nullptr) == CBS_OK);
  CHECK(cbs_bandwidth_probe(nullptr, dev, 1024, 1, nullptr, ms) == CBS_E_INVALID);
  CHECK(cbs_bandwidth_probe(dev, dev, 1000, 1, nullptr, ms) == CBS_E_INVALID);
  CHECK(cbs_bandwidth_probe(dev, dev, 1024, 0, nullptr, ms) == CBS_E_INVALID);

  // the allocation-free solve rejects before any device call
  const int pml0[3] = {0, 0, 0};
  CHECK(cbs_solve_static(275, 275, 315, d, lam, 1.0, pml0, dev, CBS_F32, &src, dev, &o, &st,
                         nullptr) == CBS_E_WORKSPACE);
  CHECK(cbs_solve_static(1, 8, 8, d, lam, 1.0, pml0, dev, CBS_F32, &src, dev, &o, &st,
                         nullptr) == CBS_E_INVALID);
  cbs_opts bo = o;
  bo.max_iter = 0;
  CHECK(cbs_solve_static(8, 8, 12, d, lam, 1.0, pml, dev, CBS_F32, &src, dev, &bo, &st,
                         nullptr) == CBS_E_INVALID);
  CHECK(cbs_solve_static(8, 8, 12, d, lam, 1.0, pml, nullptr, CBS_F32, &src, dev, &o, &st,
                         nullptr) == CBS_E_INVALID);

  // a plan laid out on the host
  HostPlan hp(8, 8, 12, pml);
  cbs_plan_s* p = &hp.plan;
  CHECK(p->ox == cbs::find_size(8) && p->oz == cbs::find_size(12) && p->nxp % kBrick == 0);
  CHECK(std::abs(p->k0 - 2 * M_PI / lam) < 1e-6 * p->k0 && p->kb == p->k0);
  CHECK(cbs_plan_set_pml_profile(p, 0, 1.0) == CBS_E_INVALID);
  CHECK(cbs_plan_set_pml_profile(p, 9, 1.0) == CBS_E_INVALID);
  CHECK(cbs_plan_set_pml_profile(p, 2, -1.0) == CBS_E_INVALID);
  CHECK(cbs_plan_set_pml_profile(p, 2, NAN) == CBS_E_INVALID);
  CHECK(cbs_plan_set_pml_profile(p, 2, INFINITY) == CBS_E_INVALID);
  CHECK(cbs_plan_set_pml_profile(p, 3, 0.5) == CBS_OK && p->order == 3 && p->sigma_max == 0.5);
  CHECK(cbs_plan_set_shift_factor(p, 0.99) == CBS_E_INVALID);
  CHECK(cbs_plan_set_shift_factor(p, NAN) == CBS_E_INVALID);
  CHECK(cbs_plan_set_shift_factor(p, 1.25) == CBS_OK && p->shift_factor == 1.25);
  CHECK(cbs_set_permittivity(p, nullptr, CBS_F32) == CBS_E_INVALID);
  CHECK(cbs_set_permittivity(p, dev, 7) == CBS_E_INVALID);
  CHECK(cbs_eps_shift(p) == -1.0);
  CHECK(cbs_history(p, hist, 4) == 0);
  // no permittivity yet: every solve is out of order
  CHECK(cbs_solve(p, &src, dev, &o, &st) == CBS_E_STATE);
  CHECK(cbs_adjoint_solve(p, dev, &src, dev, &o, &st) == CBS_E_STATE);
  CHECK(cbs_solve_begin(p, 0, nullptr, &src, dev, &o) == CBS_E_STATE);
  CHECK(cbs_solve_advance(p, 1) == CBS_E_STATE);
  CHECK(cbs_apply_green(p, dev, (char*)dev + 1) == CBS_E_STATE);
  CHECK(cbs_time_passes(p, dev, 1, ms) == CBS_E_STATE);
  CHECK(cbs_solve_batch(p, 1, &src, dev, &o, &st, dev, 1 << 30) == CBS_E_STATE);
  CHECK(cbs_solve_scpml(p, &src, dev, &o, &layer, &st, dev, 1 << 30) == CBS_E_STATE);
  // boxes and figures
  const int bad_lo[3] = {-1, 0, 0}, bad_hi[3] = {8, 9, 12}, rev_lo[3] = {4, 0, 0},
            rev_hi[3] = {3, 8, 12};
  CHECK(cbs_gradient(p, dev, dev, bad_lo, hi, 1.0, (float*)dev) == CBS_E_INVALID);
  CHECK(cbs_gradient(p, dev, dev, lo, bad_hi, 1.0, (float*)dev) == CBS_E_INVALID);
  CHECK(cbs_gradient(p, dev, dev, rev_lo, rev_hi, 1.0, (float*)dev) == CBS_E_INVALID);
  CHECK(cbs_gradient(p, nullptr, dev, lo, hi, 1.0, (float*)dev) == CBS_E_INVALID);
  CHECK(cbs_gradient(p, dev, dev, lo, lo, 1.0, (float*)dev) == CBS_OK);   // empty box: no work
  CHECK(cbs_lens_metrics(p, dev, lo, lo, 3.0, 1e-5, 1.0, &fig) == CBS_E_INVALID);
  CHECK(cbs_lens_metrics(p, dev, lo, hi, 0.0, 1e-5, 1.0, &fig) == CBS_E_INVALID);
  CHECK(cbs_lens_metrics(p, dev, lo, hi, 3.0, NAN, 1.0, &fig) == CBS_E_INVALID);
  CHECK(cbs_lens_metrics(p, dev, lo, hi, 3.0, 1e-5, -1.0, &fig) == CBS_E_INVALID);
  CHECK(cbs_lens_metrics(p, dev, lo, bad_hi, 3.0, 1e-5, 1.0, &fig) == CBS_E_INVALID);
  CHECK(cbs_tfsf_source(p, &src, lo, lo, dev) == CBS_E_INVALID);
  CHECK(cbs_tfsf_source(p, &src, bad_lo, hi, dev) == CBS_E_INVALID);
  cbs_source pt{};
  pt.kind = CBS_SRC_POINT;
  CHECK(cbs_tfsf_source(p, &pt, lo, hi, dev) == CBS_E_INVALID);
  cbs_source obl{};
  obl.kind = CBS_SRC_PLANE_WAVE;
  obl.dir[0] = 0.8;
  obl.dir[1] = 0.7;
  CHECK(cbs_tfsf_source(p, &obl, lo, hi, dev) == CBS_E_INVALID);
  // the stretched layer's parameters (the plan has a graded potential until sigma_max = 0)
  CHECK(cbs_scpml_operator(p, nullptr, dev, (char*)dev + 1, dev, 1 << 30) == CBS_E_INVALID);
  CHECK(cbs_scpml_operator(p, &layer, dev, dev, dev, 1 << 30) == CBS_E_INVALID);   // aliasing
  const cbs_scpml bad_layers[] = {{-1.0, 1, 8}, {NAN, 1, 8}, {INFINITY, 1, 8}, {0.75, 0, 8},
                                  {0.75, 9, 8}};
  for (const cbs_scpml& bl : bad_layers)
    CHECK(cbs_scpml_operator(p, &bl, dev, (char*)dev + 1, aligned, 1 << 30) == CBS_E_INVALID);
  CHECK(cbs_scpml_operator(p, &layer, dev, (char*)dev + 1, nullptr, 1 << 30) == CBS_E_WORKSPACE);
  CHECK(cbs_scpml_operator(p, &layer, dev, (char*)dev + 1, aligned + 8, 1 << 30) ==
        CBS_E_WORKSPACE);
  CHECK(cbs_scpml_operator(p, &layer, dev, (char*)dev + 1, aligned, 512) == CBS_E_WORKSPACE);

  // with a permittivity recorded: options, sources and workspaces
  p->have_eps = true;
  p->eps = 1.0;
  CHECK(cbs_solve_scpml(p, &src, dev, &o, &layer, &st, aligned, 1 << 30) == CBS_E_STATE);
  p->sigma_max = 0.0;
  cbs_opts warm = o;
  warm.flags = CBS_WARM_START;
  CHECK(cbs_solve_scpml(p, &src, dev, &warm, &layer, &st, aligned, 1 << 30) == CBS_E_INVALID);
  CHECK(cbs_solve_scpml(p, &src, dev, &o, nullptr, &st, aligned, 1 << 30) == CBS_E_INVALID);
  const cbs_scpml long_restart{0.75, 1, kScpmlMaxRestart + 1};
  CHECK(cbs_solve_scpml(p, &src, dev, &o, &long_restart, &st, aligned, 1 << 30) ==
        CBS_E_INVALID);
  CHECK(cbs_solve_scpml(p, &src, dev, &o, &layer, &st, aligned, 512) == CBS_E_WORKSPACE);
  CHECK(cbs_solve_scpml(p, &src, nullptr, &o, &layer, &st, aligned, 1 << 30) == CBS_E_INVALID);
  const cbs_opts bad_opts[] = {{1e-4, 0, 10, 0}, {1e-4, 10, 0, 0}, {-1.0, 10, 10, 0},
                               {NAN, 10, 10, 0}};
  for (const cbs_opts& b : bad_opts) {
    CHECK(cbs_solve(p, &src, dev, &b, &st) == CBS_E_INVALID);
    CHECK(cbs_solve_batch(p, 1, &src, dev, &b, &st, aligned, 1 << 30) == CBS_E_INVALID);
  }
  CHECK(cbs_solve(p, &src, dev, nullptr, &st) == CBS_E_INVALID);
  CHECK(cbs_solve(p, &src, nullptr, &o, &st) == CBS_E_INVALID);
  CHECK(cbs_solve_advance(p, 1) == CBS_E_STATE);   // nothing begun
  CHECK(cbs_solve_end(p, &st) == CBS_E_STATE);
  cbs_plan_t one[1] = {p};
  CHECK(cbs_batch_step(one, 1, 1, &done) == CBS_E_STATE);
  CHECK(cbs_apply_green(p, dev, dev) == CBS_E_INVALID);
  CHECK(cbs_apply_green(p, nullptr, dev) == CBS_E_INVALID);
  CHECK(cbs_time_passes(p, dev, 0, ms) == CBS_E_INVALID);
  CHECK(cbs_solve_batch(p, 0, &src, dev, &o, &st, aligned, 1 << 30) == CBS_E_INVALID);
  CHECK(cbs_solve_batch(p, kMaxIllum + 1, &src, dev, &o, &st, aligned, 1 << 30) ==
        CBS_E_INVALID);
  CHECK(cbs_solve_batch(p, 1, &src, dev, &o, &st, nullptr, 1 << 30) == CBS_E_WORKSPACE);
  CHECK(cbs_solve_batch(p, 1, &src, dev, &o, &st, aligned + 8, 1 << 30) == CBS_E_WORKSPACE);
  CHECK(cbs_solve_batch(p, 1, &src, dev, &o, &st, aligned, 256) == CBS_E_WORKSPACE);
  cbs_source two[2] = {src, pt};
  two[0].kind = CBS_SRC_PLANE_WAVE;
  CHECK(cbs_solve_batch(p, 2, two, dev, &o, &st, aligned, 1 << 30) == CBS_E_INVALID);

  // source set-up (no device work)
  CbsArgs a;
  Kvec kv;
  cbs_source s{};
  s.kind = 17;
  CHECK(prepare(p, 0, &s, dev, &o, a, kv) == CBS_E_INVALID);
  s.kind = CBS_SRC_FIELD;
  CHECK(prepare(p, 0, &s, dev, &o, a, kv) == CBS_E_INVALID);   // no field pointer
  s.kind = CBS_SRC_POINT;
  const int r0s[][3] = {{-1, 0, 0}, {8, 0, 0}, {0, 8, 0}, {0, 0, 12}, {0, 0, -5}};
  for (const auto& r : r0s) {
    std::memcpy(s.r0, r, sizeof(s.r0));
    CHECK(prepare(p, 0, &s, dev, &o, a, kv) == CBS_E_INVALID);
  }
  s.r0[0] = 7;
  s.r0[1] = 0;
  s.r0[2] = 11;
  CHECK(prepare(p, 0, &s, dev, &o, a, kv) == CBS_OK);
  CHECK(a.src == SRC_POINT && a.r0x == 7 && a.r0y == 0 && a.r0z == 11 && a.E == dev);
  CHECK(prepare(p, 1, &s, dev, &o, a, kv) == CBS_OK);            // adjoint point source
  CHECK(prepare(p, 1, nullptr, dev, &o, a, kv) == CBS_E_INVALID);
  s.kind = CBS_SRC_PLANE_WAVE;
  CHECK(prepare(p, 1, &s, dev, &o, a, kv) == CBS_E_INVALID);     // adjoint of a plane wave
  const double dirs[][2] = {{1.0, 0.0}, {0.8, 0.7}, {NAN, 0.0}, {0.0, -INFINITY}};
  for (const auto& dd : dirs) {
    s.dir[0] = dd[0];
    s.dir[1] = dd[1];
    CHECK(prepare(p, 0, &s, dev, &o, a, kv) == CBS_E_INVALID);
  }
  s.dir[0] = s.dir[1] = 0.0;
  CHECK(prepare(p, 0, nullptr, dev, &o, a, kv) == CBS_OK && a.src == SRC_PLANE && !a.oblique);
  CHECK(kv.pol[0][0][0] == 1.0 && kv.kd[0][0] == 0.0 &&
        std::abs(kv.kd[0][2] - p->kb * p->pitch) < 1e-15);
  s.dir[0] = 0.3;
  s.dir[1] = -0.4;
  s.pol[1][1] = 1.0;   // i y-polarised
  CHECK(prepare(p, 0, &s, dev, &o, a, kv) == CBS_OK && a.oblique);
  const double kbd = p->kb * p->pitch;
  CHECK(std::abs(kv.kd[0][0] - 0.3 * kbd) < 1e-15 && std::abs(kv.kd[0][1] + 0.4 * kbd) < 1e-15);
  CHECK(std::abs(kv.kd[0][2] - kbd * std::sqrt(0.75)) < 1e-15);
  CHECK(kv.pol[0][0][0] == 0.0 && kv.pol[0][1][1] == 1.0);
  s.kind = CBS_SRC_FIELD_CONJ;
  s.field = dev;
  CHECK(prepare(p, 1, &s, dev, &o, a, kv) == CBS_OK && a.src == SRC_FIELD_CONJ && a.fin == dev);
  s.kind = CBS_SRC_NONE;
  CHECK(prepare(p, 0, &s, dev, &o, a, kv) == CBS_OK && a.src == SRC_NONE);
  CHECK(prepare(p, 1, &s, dev, &o, a, kv) == CBS_E_INVALID);     // adjoint needs a source
}

void fwhm_checks() {
  // a triangle of half-width w is piecewise linear: the interpolated width is exact
  for (int w = 2; w <= 9; ++w)
    for (int n : {2 * w + 3, 4 * w + 7}) {
      std::unique_ptr<double[]> v(new double[n]);
      const int i0 = n / 2;
      for (int i = 0; i < n; ++i) v[i] = std::max(0.0, 1.0 - std::abs(i - i0) / double(w));
      CHECK(std::abs(fwhm_of(v.get(), n, i0, 0.25) - 0.25 * w) < 1e-12);
    }
  // a sampled Gaussian: 2 sqrt(2 ln 2) sigma to the interpolation's accuracy
  {
    const int n = 201, i0 = 97;
    const double sig = 12.5;
    std::unique_ptr<double[]> v(new double[n]);
    for (int i = 0; i < n; ++i) v[i] = std::exp(-0.5 * (i - i0) * (i - i0) / (sig * sig));
    const double f = fwhm_of(v.get(), n, i0, 1.0);
    CHECK(std::abs(f - 2.0 * std::sqrt(2.0 * std::log(2.0)) * sig) < 2e-3 * f);
  }
  // no crossing inside the profile: NaN, and no read outside [0, n)
  {
    std::unique_ptr<double[]> v(new double[1]);
    v[0] = 1.0;
    CHECK(std::isnan(fwhm_of(v.get(), 1, 0, 1.0)));
    std::unique_ptr<double[]> u(new double[6]);
    const double flat[6] = {0.2, 0.9, 1.0, 0.9, 0.8, 0.7};
    std::memcpy(u.get(), flat, sizeof(flat));
    CHECK(std::isnan(fwhm_of(u.get(), 6, 2, 1.0)));   // stays above half on the right
    CHECK(std::isnan(fwhm_of(u.get(), 6, 0, 1.0)));   // peak at the edge
  }
}

// No GPU: plan creation and the allocation-free solve fail at their first HIP
// call and leave nothing behind (the leak checker runs at exit).
void no_device_checks() {
  int count = 0;
  if (hipGetDeviceCount(&count) == hipSuccess && count > 0) {
    std::printf("a GPU is present: the no-device checks are skipped\n");
    return;
  }
  const int pml[3] = {2, 2, 3};
  const double lam = 1.064e-6, d = lam / 8;
  const size_t need = cbs_plan_workspace_bytes(8, 8, 12);
  void* ws = std::aligned_alloc(256, (need + 255) / 256 * 256);
  cbs_plan_t h = reinterpret_cast<cbs_plan_t>(0x1);
  for (int rep = 0; rep < 3; ++rep) {
    CHECK(cbs_plan_create(&h, 8, 8, 12, d, lam, 1.0, pml, ws, need, nullptr) == CBS_E_HIP);
    CHECK(h == nullptr && std::strlen(cbs_last_error()) > 0);
  }
  std::free(ws);
  cbs_opts o{1e-4, 10, 10, 0};
  cbs_stats st{};
  static unsigned char fake[1];
  CHECK(cbs_solve_static(8, 8, 12, d, lam, 1.0, pml, fake, CBS_F32, nullptr, fake, &o, &st,
                         nullptr) == CBS_E_HIP);
}

}  // namespace

int main() {
  const std::vector<int> sizes = registry_checks();
  twiddle_checks(sizes);
  layout_checks(sizes);
  argument_checks();
  fwhm_checks();
  no_device_checks();
  if (g_failed) {
    std::printf("%d of %d host checks failed\n", g_failed, g_checks);
    return 1;
  }
  std::printf("host checks passed (%d checks, %zu registered lengths)\n", g_checks,
              sizes.size());
  return 0;
}
