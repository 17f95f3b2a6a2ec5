/*
 * cbs.h -- C ABI of the MI355X (gfx950) vector convergent Born series solver.
 *
 * The library solves the 3D vector Helmholtz (Maxwell) problem of arXiv
 * 2506.15411 (simulation-setup paragraph: CBS of its references [25] and [26],
 * absorbing layer of reference [31]; design paragraph: x-polarised plane wave
 * at normal incidence) and the adjoint problem used for its permittivity
 * gradient (objective and optimisation paragraphs, Fig. 2):
 *
 *     (L - K) E_s = S,   L = F^-1 diag(|p|^2 I - pt pt^T) F,
 *     K = k0^2 eps_r + i kb^2 sigma,  kb = k0 n_bg,
 *
 * by the iteration  E_s <- E_s + gamma [G (V E_s + S) - E_s]  with
 * V = K - kb^2 - i eps, gamma = (i/eps) V, eps = kappa max|K - kb^2| (kappa >= 1,
 * the convergence condition of reference [25] being eps >= max|K - kb^2|) and
 * G^(p) = (|p|^2 I - pt pt^T - (kb^2 + i eps) I)^-1 applied by FFT.
 * pt equals p except at the Nyquist bin of an even axis, where it is 0.
 *
 * Conventions shared by every entry point
 *   - time dependence exp(-i w t); Im eps_r >= 0 (passive media only);
 *   - a grid of nx * ny * nz voxels with one pitch d; voxel (i, j, k) is
 *     centred at (i d, j d, k d);
 *   - scalar volumes are [nz][ny][nx] (x fastest); vector fields are
 *     complex64 (interleaved re, im) [3][nz][ny][nx], component 0 = x;
 *   - every pointer named *_dev is device memory (HBM) owned by the caller
 *     and borrowed for the duration of the call; the library never allocates
 *     device memory: all scratch lives in the caller's workspace;
 *   - all work is ordered on the HIP stream given at plan creation;
 *   - functions return a cbs_status; cbs_last_error() describes the last
 *     non-OK status of the calling thread.
 *   - a plan is used by one host thread at a time; distinct plans (with
 *     distinct workspaces) may run concurrently.
 */
#ifndef CBS_H
#define CBS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cbs_plan_s* cbs_plan_t;

typedef enum {
  CBS_OK = 0,
  CBS_NOT_CONVERGED = 1,   /* max_iter reached; the output holds the last iterate */
  CBS_E_INVALID = -1,      /* bad argument, inadmissible medium, unsupported size  */
  CBS_E_WORKSPACE = -2,    /* workspace missing, misaligned or too small          */
  CBS_E_HIP = -3,          /* a HIP runtime call failed                            */
  CBS_E_DIVERGED = -4,     /* non-finite residual                                  */
  CBS_E_STATE = -5         /* call out of order (e.g. solve before permittivity)   */
} cbs_status;

enum { CBS_F32 = 0, CBS_C64 = 1 };   /* permittivity dtype */

enum {
  CBS_SRC_NONE = 0,        /* S = 0 */
  CBS_SRC_PLANE_WAVE = 1,  /* S = k0^2 (eps_r - n_bg^2) pol exp(i k.r), k towards +z     */
  CBS_SRC_FIELD = 2,       /* S = field (device complex64 [3][nz][ny][nx], units 1/m^2) */
  CBS_SRC_POINT = 3,       /* S = amp at voxel r0, zero elsewhere (units 1/m^2)        */
  CBS_SRC_FIELD_CONJ = 4   /* S = conj(field), field as for FIELD: the adjoint source
                              conj(gE) of a loss whose derivative gE = 2 dL/dE* is held
                              in device memory (optimisation paragraph: the gradient
                              through one more CBS solve); conjugated on the device   */
};

enum {
  CBS_WARM_START = 1u,        /* E_dev holds the initial iterate (total field for a
                                 plane-wave solve, adjoint field for an adjoint solve) */
  CBS_RETURN_SCATTERED = 2u,  /* plane-wave solve: return E_s instead of E_inc + E_s */
  CBS_RECORD_HISTORY = 4u     /* keep the residual of every iteration (cbs_history) */
};

typedef struct {
  double tol;          /* stop when ||E^(k+1) - E^(k)|| / ||E^(k+1)|| <= tol (FP64 norms) */
  int max_iter;        /* hard cap on iterations (>= 1)                                   */
  int check_every;     /* host polls the device convergence flag every this many
                          iterations (>= 1); iterations past convergence are skipped on
                          the device, so this only trades host syncs for idle launches   */
  unsigned flags;      /* CBS_WARM_START | CBS_RETURN_SCATTERED | CBS_RECORD_HISTORY      */
} cbs_opts;

typedef struct {
  int iterations;      /* updates applied                                  */
  int converged;       /* 1 if the residual reached tol                    */
  double residual;     /* last relative update norm (FP64)                 */
  double eps_shift;    /* eps in 1/m^2                                     */
  float ms;            /* device time of the iteration loop (HIP events)   */
} cbs_stats;

typedef struct {
  int kind;                 /* CBS_SRC_*                                              */
  double pol[3][2];         /* PLANE_WAVE: polarisation (re, im) per component;
                               all zero means x-polarised (the design paragraph's
                               illumination); the caller keeps it transverse to k    */
  const void* field;        /* FIELD, FIELD_CONJ: device complex64 [3][nz][ny][nx]    */
  int r0[3];                /* POINT: voxel (ix, iy, iz)                              */
  double amp[3][2];         /* POINT: amplitude (re, im) per component                */
  double dir[2];            /* PLANE_WAVE: transverse direction cosines (sx, sy) =
                               (kx, ky) / kb with sx^2 + sy^2 < 1, kz = kb sqrt(1 -
                               sx^2 - sy^2) > 0; (0, 0) is normal incidence.  The
                               incident wave is pol exp(i k.r), phase 0 at voxel
                               (0, 0, 0).  Zero-initialise for normal incidence.     */
} cbs_source;

/* Device bytes a plan of this grid needs as workspace (exact). 0 if the grid
 * is not supported (see cbs_axis_supported). */
size_t cbs_plan_workspace_bytes(int nx, int ny, int nz);

/* 1 if n is a supported length for axis 0 = x, 1 = y, 2 = z, else 0.
 * The FFT passes are specialised per length (two-level splits n = n1 * n2
 * with register codelets for radices 2..37). */
int cbs_axis_supported(int axis, int n);

/* Create a plan.
 *   nx, ny, nz     grid (each >= 2 and supported on its axis)
 *   pitch_m        voxel pitch d > 0 (metres)
 *   lambda0_m      vacuum wavelength > 0 (metres)
 *   n_bg           background index > 0 (real)
 *   pml            per-side absorbing-layer thickness in voxels, 0 <= 2 pml[a] < n[a]
 *   workspace_dev  caller device memory, >= cbs_plan_workspace_bytes, 256-byte aligned,
 *                  must outlive the plan
 *   stream         hipStream_t the plan's work is ordered on (NULL = default stream)
 * The absorbing profile defaults to sigma = 1 * min(1, sum_a u_a^2), u_a the depth
 * into the layer in units of its thickness (outermost voxel u = 1). */
int cbs_plan_create(cbs_plan_t* out, int nx, int ny, int nz, double pitch_m,
                    double lambda0_m, double n_bg, const int pml[3],
                    void* workspace_dev, size_t workspace_bytes, void* stream);

/* Change the absorbing profile: sigma = sigma_max * min(1, sum_a u_a^order).
 * Must precede cbs_set_permittivity (it invalidates the potential). */
int cbs_plan_set_pml_profile(cbs_plan_t plan, int order, double sigma_max);

/* Set eps = kappa * max|K - kb^2| (kappa >= 1, default 1.1).  Every admissible
 * eps gives the same converged field; kappa slightly above 1 damps the high
 * spatial frequencies of the strongest-contrast voxels, which kappa = 1 leaves
 * undamped (local factor |V0|/eps = 1).  Must precede cbs_set_permittivity. */
int cbs_plan_set_shift_factor(cbs_plan_t plan, double kappa);

/* Set the medium: eps_r_dev is [nz][ny][nx] float32 (CBS_F32) or complex64
 * (CBS_C64).  Validates finiteness, Im eps_r >= 0 and eps_r == n_bg^2 (at
 * float32) inside the absorbing layer, builds the potential on the device and
 * computes eps = kappa max|K - kb^2| with the maximum taken in FP64 (floor
 * 1e-3 kb^2 on the maximum).  Returns CBS_E_INVALID for a medium that fails
 * these checks or whose eps d^2 reaches 1e30 (the FP32 iteration would
 * overflow).  Synchronises the stream. */
int cbs_set_permittivity(cbs_plan_t plan, const void* eps_r_dev, int dtype);

/* Forward solve.  src = NULL means an x-polarised plane wave.  E_dev is
 * complex64 [3][nz][ny][nx]: on return the total field E_inc + E_s for a
 * plane-wave source (E_s with CBS_RETURN_SCATTERED), or the solution of
 * A E = S for FIELD/POINT/NONE sources.  Synchronises the stream.
 * Returns CBS_OK, CBS_NOT_CONVERGED (valid last iterate) or an error. */
int cbs_solve(cbs_plan_t plan, const cbs_source* src, void* E_dev,
              const cbs_opts* opts, cbs_stats* stats);

/* Adjoint solve with the same operator (A is complex-symmetric, so the
 * adjoint field of a real objective is E_adj = A^-1 g with g the conjugated
 * derivative of the objective).
 *   adj_src POINT with E_fwd_dev != NULL: g = conj(E_fwd(r0)) at r0, built on
 *           the device (gradient of |E(r0)|^2 with scale 2 in cbs_gradient);
 *   adj_src POINT with E_fwd_dev == NULL: g = adj_src->amp at r0;
 *   adj_src FIELD: g = adj_src->field;
 *   adj_src FIELD_CONJ: g = conj(adj_src->field).
 * E_adj_dev receives complex64 [3][nz][ny][nx].  Synchronises the stream. */
int cbs_adjoint_solve(cbs_plan_t plan, const void* E_fwd_dev, const cbs_source* adj_src,
                      void* E_adj_dev, const cbs_opts* opts, cbs_stats* stats);

/* ---- asynchronous solves (continuous batching) --------------------------
 * The blocking cbs_solve / cbs_adjoint_solve are built from these.  A plan
 * holds at most one solve in progress; solves on distinct plans (each with its
 * own stream) overlap on the device.  Every call returns without waiting for
 * the device except cbs_solve_end and cbs_batch_step.
 *
 * Begin a forward (adjoint = 0; arguments as cbs_solve) or adjoint (adjoint = 1;
 * arguments as cbs_adjoint_solve) solve: validates, initialises the device state
 * and enqueues the prologue. */
int cbs_solve_begin(cbs_plan_t plan, int adjoint, const void* E_fwd_dev, const cbs_source* src,
                    void* E_dev, const cbs_opts* opts);

/* Enqueue up to `iters` more iterations (never past opts->max_iter) followed by
 * an asynchronous copy of the device state; iterations after the device has
 * stopped return at once.  At most 4 quanta may be outstanding
 * (CBS_E_STATE beyond that: poll first). */
int cbs_solve_advance(cbs_plan_t plan, int iters);

/* Retire completed quanta without waiting; *done = 1 once the device has
 * stopped (converged, max_iter reached or diverged); *outstanding (may be
 * NULL) receives the number of quanta still in flight. */
int cbs_solve_poll(cbs_plan_t plan, int* done, int* outstanding);

/* Wait for outstanding quanta, enqueue the final E_inc addition of a plane-wave
 * solve, fill stats and return the solve's status (CBS_OK, CBS_NOT_CONVERGED or
 * CBS_E_DIVERGED).  CBS_E_STATE if the device has not stopped yet.  The field is
 * complete when the plan's stream reaches this point. */
int cbs_solve_end(cbs_plan_t plan, cbs_stats* stats);

/* ---- batched illuminations -----------------------------------------------
 * Several plane-wave illuminations of one medium solved together (multi-angle
 * or multi-polarisation illumination; the paper's design uses one x-polarised
 * normal-incidence wave, design paragraph).  One launch of each pass advances
 * all of them: the potential is read once per row for all illuminations and
 * small grids need a fraction of the launches.  Every illumination has its own
 * residual; the solve stops when the largest reaches tol (or at max_iter), so
 * all illuminations run the same number of iterations, and at equal iteration
 * counts each field equals a cbs_solve of that source alone (bit for bit when
 * the batch's illuminations are all at normal incidence or all oblique; a
 * normal-incidence wave batched with an oblique one runs the x pass compiled
 * for oblique waves and agrees to FP32 rounding).
 *
 * Device bytes of the batch workspace for `count` illuminations (1..8): the
 * spectral work fields, residual partials and phase tables of the batch; 0 if
 * the grid is not supported or count is out of range. */
size_t cbs_batch_workspace_bytes(int nx, int ny, int nz, int count);

/* Solve `count` (1..8) PLANE_WAVE sources srcs[0..count) on the plan's medium.
 *   E_dev      complex64 [count][3][nz][ny][nx]: total fields (scattered with
 *              CBS_RETURN_SCATTERED); with CBS_WARM_START it holds initial
 *              iterates (total fields)
 *   stats      count entries: the shared iteration count, each illumination's
 *              last residual and whether it is <= tol
 *   work_dev   device memory of >= cbs_batch_workspace_bytes, 256-byte aligned,
 *              owned by the caller (the plan's own spectral field is not used)
 * Returns CBS_OK when every illumination met tol, CBS_NOT_CONVERGED at max_iter,
 * or an error.  Synchronises the plan's stream. */
int cbs_solve_batch(cbs_plan_t plan, int count, const cbs_source* srcs, void* E_dev,
                    const cbs_opts* opts, cbs_stats* stats, void* work_dev, size_t work_bytes);

/* Grouped step: enqueue `iters` iterations on every plan (each on its own
 * stream, so their work overlaps), then wait for all of them; done_out[i] = 1
 * for plans whose solve has stopped.  Every plan must have a solve begun. */
int cbs_batch_step(cbs_plan_t* plans, int count, int iters, int* done_out);

/* ---- stretched-coordinate absorbing layer -------------------------------
 * The paper bounds its volume with a perfectly matched layer after its
 * reference [31] (simulation-setup paragraph), a stretched-coordinate PML.  Here every
 * derivative d/da inside the layer of axis a becomes (1/s_a) d/da with
 * s_a = 1 + i alpha_max u_a^order (u_a the depth into the layer in units of its
 * thickness, outermost voxel u = 1, the same u as the graded potential's), on the
 * solver's spectral derivatives.  The system (L_s - k0^2 eps_r) E_s = S is not a
 * CBS splitting (the stretched derivatives are not a bounded potential), so it is
 * solved by restarted GMRES on the CBS-preconditioned form
 *     gamma [E_s - G (V E_s - (L_s - L) E_s)] = gamma G S
 * whose operator is one CBS iteration with the field source -(L_s - L) E_s plus
 * the per-axis stretched-derivative products.  The plan must have no graded
 * potential (cbs_plan_set_pml_profile(plan, order, 0) before
 * cbs_set_permittivity): the stretched layer replaces it. */
typedef struct {
  double alpha_max;   /* >= 0; 0 turns the layer off (then the solve is the plain
                         spectral problem on the periodic grid)                   */
  int order;          /* 1..8, the profile exponent                              */
  int restart;        /* GMRES restart length, 1..64 (workspace grows with it)   */
} cbs_scpml;

/* Device bytes of the stretched-layer workspace: restart + 1 basis fields, the
 * right-hand side, the stretched-derivative source, two scalar fields, the dense
 * per-axis operators (3 n_a^2 complex64 per axis) and reduction buffers.  0 if
 * the grid is not supported, an axis exceeds 1024 or restart is out of range. */
size_t cbs_scpml_workspace_bytes(int nx, int ny, int nz, int restart);

/* Solve with the stretched layer.
 *   src        as cbs_solve (plane wave, field, point or none)
 *   E_dev      complex64 [3][nz][ny][nx]: E_inc + E_s for a plane wave (E_s with
 *              CBS_RETURN_SCATTERED), E_s otherwise; overwritten from zero
 *   opts       tol: relative residual ||b - B E_s|| / ||b|| of the preconditioned
 *              system (FP64 norms, the true residual at the end of a restart
 *              cycle); max_iter: GMRES steps (one operator application each);
 *              flags: CBS_RETURN_SCATTERED, CBS_RECORD_HISTORY (cbs_history then
 *              gives the GMRES residual estimate of every step); CBS_WARM_START
 *              is rejected; check_every is ignored
 *   layer      alpha_max, order, restart
 *   stats      iterations = GMRES steps, residual = the last true residual
 *   work_dev   >= cbs_scpml_workspace_bytes(nx, ny, nz, layer->restart), 256-byte
 *              aligned, owned by the caller
 * Returns CBS_OK, CBS_NOT_CONVERGED (E_dev holds the last iterate), CBS_E_STATE
 * for a plan with a graded potential, or an error.  Synchronises the plan's
 * stream after every step (the host runs the Givens rotations). */
int cbs_solve_scpml(cbs_plan_t plan, const cbs_source* src, void* E_dev, const cbs_opts* opts,
                    const cbs_scpml* layer, cbs_stats* stats, void* work_dev, size_t work_bytes);

/* The stretched layer's addition to the operator, out = (L_s - L) in (units
 * 1/m^2), for complex64 [3][nz][ny][nx] fields in != out.  work_dev as for
 * cbs_solve_scpml with restart = 1 (layer->restart is ignored).  Asynchronous on
 * the plan's stream. */
int cbs_scpml_operator(cbs_plan_t plan, const cbs_scpml* layer, const void* in_dev,
                       void* out_dev, void* work_dev, size_t work_bytes);

/* Permittivity gradient over a half-open box [lo, hi) (x, y, z):
 *   grad[z][y][x] = scale * k0^2 * Re(sum_c E_adj,c * E_c)
 * (dK/d eps_r = k0^2; scale = 2 for the adjoint source conj(E(r0)) of
 * |E(r0)|^2, 1 for a source conj(gE) with gE = 2 dL/dE*).  grad_dev is float32,
 * box-shaped, x fastest.  Asynchronous on the plan's stream. */
int cbs_gradient(cbs_plan_t plan, const void* E_dev, const void* E_adj_dev,
                 const int box_lo[3], const int box_hi[3], double scale, float* grad_dev);

/* Lens figures of a field (focusing-efficiency paragraph: eta_f is the power in
 * a disc of diameter three lateral FWHM at the focal plane over the incident
 * power, reference [18]).  Readings: the focal point is the maximum of |E|^2
 * (summed over components) in the search box; the FWHM are those of |E|^2
 * along x and y in the focal plane and along z through the focus; the power
 * through the disc (centred on the focus, voxel centres within the radius) is
 * the flux of the Poynting vector S_z = Re(Ex conj(Hy) - Ey conj(Hx)) of the
 * plane's propagating angular spectrum (H = k x E / k per plane wave, Ez from
 * k . E = 0, evanescent components dropped; units where a plane wave of
 * amplitude e0 carries |e0|^2), and the incident power is |e0|^2 pi (D/2)^2
 * (plane wave on the aperture D in the same medium). */
typedef struct {
  int focus[3];        /* voxel (x, y, z) of the maximum of |E|^2 in the search box */
  double peak;         /* |E|^2 there                                                */
  double fwhm[3];      /* widths at half maximum along x, y in the focal plane and
                          along z on the axis through the focus (metres; linear
                          interpolation between voxels; NaN if a crossing is not
                          inside the grid)                                           */
  double disc_flux;    /* Poynting flux through the disc, m^2 x |e0|^2 (NaN if a
                          lateral fwhm is)                                           */
  double eta_f;        /* disc_flux / (|e0|^2 pi (D/2)^2) (NaN if a lateral fwhm is) */
} cbs_lens_figures;

/* Focus, FWHM and focusing efficiency of the complex64 field E_dev
 * [3][nz][ny][nx] (normally the total field of a plane-wave solve).  The
 * focus is searched in the half-open box [lo, hi) (x, y, z; ties go to the
 * smaller linear index); the disc diameter is disc_factor times the mean of
 * the x and y FWHM (3 in the paper); aperture_m is the lens diameter D and e0
 * the incident amplitude.  Plane transforms and reductions are in FP64.
 * Synchronises the plan's stream.  Uses the plan's workspace. */
int cbs_lens_metrics(cbs_plan_t plan, const void* E_dev, const int lo[3], const int hi[3],
                     double disc_factor, double aperture_m, double e0, cbs_lens_figures* out);

/* Total-field / scattered-field source of a plane wave (PLANE_WAVE src: pol
 * and direction; NULL = x-polarised normal incidence) for the box [lo, hi)
 * (x, y, z, half-open, inside the grid):
 *     S = (L - K_bg)(chi E_inc),  K_bg = kb^2 (1 + i sigma),
 * chi the box's indicator.  Used as the FIELD source of cbs_solve it injects
 * the plane wave on the box's faces: in the background medium the solution is
 * exactly chi E_inc, and with material inside the box it is the total field
 * inside the box and the scattered field outside (an alternative to the
 * volume source of the scattered-field formulation, for a lens illuminated
 * through its aperture; the paper's own solves use the plane wave of the
 * design paragraph).  Every term of L(chi E_inc) is a product of 1D spectral
 * derivatives of the box's edges, formed in FP64 (direct O(n^2) sums per axis)
 * and rounded to complex64 in S_dev [3][nz][ny][nx] (1/m^2).  Uses the plan's
 * spectral work field as scratch (CBS_E_STATE while a solve is in progress);
 * needs no permittivity.  Asynchronous on the plan's stream. */
int cbs_tfsf_source(cbs_plan_t plan, const cbs_source* src, const int lo[3], const int hi[3],
                    void* S_dev);

/* One application of the Green's operator of the current medium:
 * out = F^-1 G^(p) F in  (complex64 fields; in and out may not alias).
 * Asynchronous on the plan's stream. */
int cbs_apply_green(cbs_plan_t plan, const void* in_dev, void* out_dev);

/* Residual history of the last solve with CBS_RECORD_HISTORY: copies up to
 * max entries into host memory, returns the number available (>= 0) or an
 * error. */
int cbs_history(cbs_plan_t plan, double* out_host, int max);

/* Measurement aid: run a cold-start plane-wave solve of exactly `iters`
 * iterations (no early stop) into E_dev, with HIP events recorded on the
 * plan's stream between the passes, and return the mean device time per
 * launch in ms_out[0..4] = { y forward, z (forward + Green + inverse),
 * y inverse, x (inverse + update + forward), residual } (the residual
 * reduction normally runs inside the x pass; ms_out[4] is then 0).
 * Synchronises. */
int cbs_time_passes(cbs_plan_t plan, void* E_dev, int iters, float* ms_out);

/* Measurement aid (no plan needed): copy `bytes` (a multiple of 16) from
 * src_dev to dst_dev `reps` times with a plain streaming copy kernel on
 * `stream` and return the mean device ms per copy in *ms_out.  Used as the
 * achievable-bandwidth reference and to calibrate memory counters.
 * Synchronises the stream. */
int cbs_bandwidth_probe(const void* src_dev, void* dst_dev, size_t bytes, int reps,
                        void* stream, float* ms_out);

/* ---- allocation-free solve ----------------------------------------------
 * For callers that cannot allocate device memory or create HIP objects (code
 * under stream capture, tight serving loops, harnesses that forbid hipMalloc):
 * the forward solve of cbs_plan_create + cbs_set_permittivity + cbs_solve in
 * one call that allocates nothing (no hipMalloc, hipFree, host-pinned memory,
 * events or other allocating routine).  Its scratch -- the workspace a plan of
 * this grid would take: spectral work field, potential, tables, partial sums,
 * solve state -- is one static device array of CBS_STATIC_SCRATCH_BYTES, which
 * each GPU the library runs on holds until the process ends.
 *   nx .. pml        as cbs_plan_create (default absorbing profile, shift 1.1)
 *   eps_r_dev, dtype as cbs_set_permittivity (same validation)
 *   src .. stats     as cbs_solve; stats->ms is host wall time of the solve
 *   stream           hipStream_t the work is ordered on (NULL = default stream)
 * Returns CBS_E_WORKSPACE, before any device work, for a grid whose workspace
 * (cbs_plan_workspace_bytes) exceeds CBS_STATIC_SCRATCH_BYTES (64^3 and 128^3
 * fit; the 275 x 275 x 315 lens does not).  Synchronises the stream; the field
 * is complete on return.  Every call on a GPU uses that GPU's one array: calls
 * that overlap on one GPU (other host threads, other streams) race and must be
 * serialised by the caller.  Nothing an earlier call left in the array is read. */
#define CBS_STATIC_SCRATCH_BYTES ((size_t)96 << 20)
int cbs_solve_static(int nx, int ny, int nz, double pitch_m, double lambda0_m, double n_bg,
                     const int pml[3], const void* eps_r_dev, int dtype, const cbs_source* src,
                     void* E_dev, const cbs_opts* opts, cbs_stats* stats, void* stream);

/* eps (1/m^2) of the current medium, or a negative value if none is set. */
double cbs_eps_shift(cbs_plan_t plan);

int cbs_plan_destroy(cbs_plan_t plan);

/* Message describing the last non-OK status returned on this thread. */
const char* cbs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CBS_H */
