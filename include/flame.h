/*
 * flame.h - C ABI of the MI355X (gfx950) spectral flame-front stepper.
 *
 * The library advances the Fourier coefficients of the flame perturbation
 * Phi(theta, phi, t) of an expanding sphere of radius r0(t) = t under Eq. (1)
 * of V. Karlin, "Global communications in multiprocessor simulations of
 * flames" (Section 2):
 *
 *   dPhi~_k/dt = (-|kappa|^2/r0^2 + gamma |kappa|/(2 r0)) Phi~_k
 *                - 1/(2 r0^2) sum_l kappa_l . kappa_{k-l} Phi~_l Phi~_{k-l},
 *
 * kappa = (s1 k1, s2 k2) with s1 = s2 = theta_pi for the literal equation, no
 * forcing. The quadratic term is evaluated on the padded N1 x N2 grid the way
 * Section 3 describes (transforms of the gradient components, pointwise
 * product, inverse transforms); the retained box is |k_i| <= K_i with
 * K_i = N_i/4 - 1 (the augmented-array size rule of Section 3 with k0 = 3).
 * Time integration is integrating-factor Euler: the linear operator is
 * integrated exactly over each step, the quadratic term is explicit.
 *
 * Conventions for every entry point:
 *  - All calls return 0 (FLAME_OK) or a negative FLAME_ERR_* code; the text of
 *    the last error of the calling thread is returned by flame_last_error().
 *    No C++ exception crosses this interface.
 *  - Every pointer named "dev" is device memory on the device that was current
 *    at flame_init. The caller owns all device memory (states, workspace,
 *    input and output buffers); the plan owns only host-side metadata.
 *  - Work is queued asynchronously on the stream given to flame_init
 *    (a hipStream_t passed as void*, 0 for the null stream). Calls that only
 *    queue device work do not synchronise.
 *  - A plan is not thread-safe; use one plan per stream.
 *
 * Supported grids: N1 and N2 powers of two with 16 <= N_i <= 16384 (flame_init
 * also checks that every kernel of the grid fits the device's LDS per workgroup).
 * A 16384-point transform runs on 1024 threads of one workgroup with 16 (or,
 * for 3/4 of the length, 12) points each; 8 points per thread stop at 8192.
 *
 * State layout (internal to the stepper but documented for checkpointing):
 * complex64 S[m][s], m = k2 in [0, N2/4), s in [0, N1/2) with k1 = s - N1/4;
 * entries with s = 0 (k1 = -N1/4, outside the box) are zero. The k2 < 0
 * half follows from Phi~(-k) = conj(Phi~(k)). Size: N1*N2 bytes.
 *
 * Canonical spectrum layout (flame_set_spectrum / flame_get_spectrum):
 * complex64 half[k1 + K1][k2], shape (2 K1 + 1) x (K2 + 1), row-major;
 * the k2 = 0 column holds both signs of k1.
 */
#ifndef FLAME_H
#define FLAME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FLAME_OK 0
#define FLAME_ERR_INVALID_ARG (-1)
#define FLAME_ERR_WORKSPACE_TOO_SMALL (-2)
#define FLAME_ERR_HIP (-3)
#define FLAME_ERR_UNSUPPORTED_SIZE (-4)
#define FLAME_ERR_NONFINITE (-5)
#define FLAME_ERR_TIMEOUT (-6)

typedef struct flame_plan_s* flame_plan;

/* Problem description of one flame (Section 2: gamma = 0.8, t0 = 200 in the
 * paper's runs; theta_pi is the segment integer; dt is the fixed step). */
typedef struct {
  int32_t n1, n2;         /* physical grid, theta x phi; powers of two in [16, 16384] */
  double gamma;           /* density contrast 1 - rho_b/rho_u, >= 0 */
  double theta_pi;        /* segment integer theta_pi, > 0 */
  double t0;              /* time of step index 0, > 0 */
  double dt;              /* time step, > 0 */
  double axis_scale[2];   /* wavenumber scale per axis; {0, 0} means {theta_pi, theta_pi} */
  int32_t r0_law;         /* reference radius: 0 r0(t) = t (Section 2); 1 a table (flame_set_r0_table) */
  int32_t integrator;     /* time integrator (see flame_step): 0 integrating-factor Euler;
                             1 integrating-factor Heun. Flames of one grid are launched
                             together only when their integrators agree. */
} flame_desc;

/* Bytes of one flame's state buffer (complex64 S, see the layout above). */
int flame_state_bytes(const flame_desc* desc, size_t* bytes);

/* Bytes of workspace that flame_init needs for n_flames flames described by
 * descs[0..n_flames-1]. */
int flame_workspace_bytes(const flame_desc* descs, int32_t n_flames, size_t* bytes);

/* Create a plan for n_flames flames. states[f] (dev, flame_state_bytes each)
 * and ws (dev, ws_bytes >= flame_workspace_bytes) stay bound to the plan until
 * flame_destroy. Builds twiddle tables on the host (double precision, rounded
 * once to float) and copies them into ws on the stream. The states are not
 * initialised: call flame_set_spectrum or flame_set_state next. Fails with
 * FLAME_ERR_UNSUPPORTED_SIZE if a kernel of some flame's grid needs more LDS
 * per workgroup than the device offers (the 16384-point transforms use up to
 * 139 KB). */
int flame_init(const flame_desc* descs, int32_t n_flames, void* const* states, void* ws, size_t ws_bytes,
               void* hip_stream, flame_plan* out);

/* Load flame `flame` from the canonical half spectrum (dev, complex64, see
 * above) and set the plan's step index to n (time t0 + n dt). The k2 = 0
 * column is symmetrised: entries with k1 > 0 are copied conjugated onto
 * k1 < 0 and Im Phi~_0 is set to 0 (Section 3, symmetrisation). */
int flame_set_spectrum(flame_plan plan, int32_t flame, const void* half, int64_t n);

/* Write flame `flame`'s state in the canonical half layout (dev, complex64). */
int flame_get_spectrum(flame_plan plan, int32_t flame, void* half);

/* Project a physical field phi (dev, float32, n1 x n2 row-major, phi fastest)
 * onto the retained box: Phi~ = (1/P) DFT(phi) for |k_i| <= K_i, then
 * symmetrise. Sets the step index to n. */
int flame_set_state(flame_plan plan, int32_t flame, const float* phi, int64_t n);

/* Synthesize flame `flame`'s field on the grid into phi (dev, float32,
 * n1 x n2 row-major): Phi(x_j) = sum_k Phi~_k exp(i k.x_j). */
int flame_get_state(flame_plan plan, int32_t flame, float* phi);

/* The caller wrote the state buffer of flame `flame` directly (e.g. restored
 * a checkpoint with a device copy), or those of every flame with flame = -1:
 * set the plan's step index to n (one index for all flames) and mark the
 * intermediate arrays of that flame (or of all) stale, so the next step
 * rebuilds them (the column pass a1 of Section 3). */
int flame_state_modified(flame_plan plan, int32_t flame, int64_t n);

/* Step index of the plan (time of flame f is t0_f + index * dt_f). */
int flame_step_index(flame_plan plan, int64_t* n);

/* Advance every bound flame by nsteps steps of Eq. (1) (the paper leaves the
 * integrator to its references). With integrator 0, integrating-factor Euler:
 *   Phi~ <- E_k (Phi~ + dt (f~_k + N_k(Phi~, t_n))),
 * E_k = exp(int sigma_k dt) over the step, N_k = (1/(2 r0(t_n)^2))
 * DFT_k[|grad Phi|^2] / P on the box, f~ the bound forcing (zero by default),
 * followed by the symmetrisation of Section 3. With integrator 1,
 * integrating-factor Heun (second order): that Euler step is the predictor
 * Phi* (symmetrised, kept in the workspace), and
 *   Phi~ <- (Phi* + E_k Phi~ + dt (f~_k + N_k(Phi*, t_{n+1}))) / 2,
 * symmetrised; it runs the row and column kernels twice per step, and with
 * r0_law = 1 it also reads table entry n + 1. nsteps >= 0. */
int flame_step(flame_plan plan, int32_t nsteps);

/* Integral diagnostics of flame `flame` at the current step (the averages of
 * Section 3; <Phi_t> as plotted in Section 2), accumulated in double:
 *   out4[0] = mean radius r0(t) + Re Phi~_0,
 *   out4[1] = averaged velocity <Phi_t> = dPhi~_0/dt = sum_k |kappa|^2 |Phi~_k|^2 / (2 r0^2),
 *   out4[2] = area excess J = mean over the grid of sqrt(1 + x) - 1,
 *             x = |grad Phi|^2 / r0^2, evaluated as x / (1 + sqrt(1 + x)),
 *   out4[3] = 1 if every state entry is finite, else 0.
 * out4 is dev memory (4 doubles), written on the stream. dJ_dstate
 * (nullable, dev, the state layout): when given, also the adjoint seed
 * dJ/dPhi at the current state as a cotangent, i.e. flame_area_gradient
 * at the current step index and state; that uses the plan's workspace, so
 * the next step rebuilds the flame's intermediates. */
int flame_diagnostics(flame_plan plan, int32_t flame, double* out4, void* dJ_dstate);

/* The same averages written to host memory (host_out4, 4 doubles), for
 * callers that check a run as it goes: queues flame_diagnostics (no seed) into the
 * plan's workspace, copies the result and waits for the plan's stream.
 * Returns FLAME_ERR_NONFINITE (with host_out4 filled) when some state entry
 * is not finite, FLAME_OK otherwise. */
int flame_diagnostics_host(flame_plan plan, int32_t flame, double* host_out4);

/* Adjoint of one step (integrating-factor Euler; the paper has no adjoint).
 * Cotangents are the Fourier coefficients of the gradient with respect to the
 * grid values of Phi, in the state layout (dev, complex64, flame_state_bytes):
 * for band-limited real fields a, b the pairing is the grid sum
 * sum_j a(x_j) b(x_j) = P Re sum_k conj(a~_k) b~_k over the whole box.
 * For the step n -> n+1 taken from state_n (the state at step index n):
 *   lam_out = mu - 2 dt c_n Pi div(m grad Phi^n),  mu = E^n lam_in,
 * m the grid field of mu, c_n = 1/(2 r0(t_n)^2). lam_out may equal lam_in;
 * state_n must not alias lam_out. Runs on the grid flame_step uses for this
 * flame (see flame_set_product_grid: the transpose of that step). Uses the
 * plan's workspace, so the next flame_step rebuilds its intermediates. It is
 * the transpose of integrating-factor Euler: a flame with integrator 1 gets
 * FLAME_ERR_INVALID_ARG. */
int flame_adjoint_step(flame_plan plan, int32_t flame, int64_t n, const void* state_n, const void* lam_in,
                       void* lam_out);

/* Gradient of the area excess J of flame_diagnostics at step index n with
 * respect to the grid values of Phi, evaluated at `state` (dev, state layout),
 * written as a cotangent (see flame_adjoint_step):
 *   lam_out = -Pi div( grad Phi / (P r0^2 sqrt(1 + |grad Phi|^2 / r0^2)) ). */
int flame_area_gradient(flame_plan plan, int32_t flame, int64_t n, const void* state, void* lam_out);

/* Reference-radius table of flame `flame` (r0_law = 1): `table` (dev, FP64,
 * caller-owned, n_entries x 3, entry n = {r0(t_n), I1_n, I2_n} with
 * t_n = t0 + n dt, I1_n = int_{t_n}^{t_{n+1}} ds / r0(s) and
 * I2_n = int ds / r0(s)^2) gives the coefficients of Eq. (1) at step n:
 * c_n = 1/(2 r0(t_n)^2), the exact linear propagator
 * exp(-|kappa|^2 I2_n + gamma |kappa| I1_n / 2), and r0 for the diagnostics.
 * It stays bound until replaced or flame_destroy. A step, adjoint step or
 * diagnostic at step index n needs n < n_entries; calls that would go beyond
 * the table, or reach a flame with r0_law = 1 and no table, fail with
 * FLAME_ERR_INVALID_ARG before launching anything. */
int flame_set_r0_table(flame_plan plan, int32_t flame, const double* table, int64_t n_entries);

/* Forcing f~_k(t) of Eq. (1) (Section 2; zero in the paper's runs) for flame
 * `flame`: `forcing` (dev, complex64, caller-owned, flame_state_bytes, in the
 * state layout above) holds f~_k for the stored half of the box, or is null
 * for no forcing (the default). Each step n -> n+1 then takes it explicitly,
 * inside the propagator like the quadratic term:
 *   Phi~^{n+1} = E (Phi~^n + dt (f~ - c_n N(Phi~^n))),
 * before the k2 = 0 column is symmetrised, so its k1 < 0 entries and
 * Im f~_0 have no effect; entries outside the box are ignored. The buffer is
 * read by every later step until replaced or flame_destroy: for a forcing
 * that varies in time, rewrite it (stream-ordered) between calls of
 * flame_step, which then uses one forcing for all of its nsteps steps (with
 * integrator 1, for both of Heun's stages, i.e. also as f~(t_{n+1}); a
 * forcing that varies within a step is then taken to first order only). The
 * adjoint and gradient calls do not depend on it. A grid-size group steps
 * with a column-kernel variant that reads the forcing while any of its
 * flames has one bound (members without one are stepped unforced by it);
 * binding the first or removing the last forcing of a group rebuilds the
 * step graph at the next flame_step. Waits for the plan's stream. Fails with
 * FLAME_ERR_INVALID_ARG for a pointer not 8-byte aligned. */
int flame_set_forcing(flame_plan plan, int32_t flame, const void* forcing);

/* Grid field of any spectrum in the state layout (a state or a cotangent):
 * phi(x_j) = sum_k spec~_k exp(i k.x_j) (dev, float32, n1 x n2 row-major). */
int flame_synthesize(flame_plan plan, int32_t flame, const void* spec, float* phi);

/* Start timing every kernel launch that flame_step and flame_diagnostics
 * queue from now on (benchmarking aid). The row and column step kernels that
 * flame_step launches directly carry a start and a stop HIP event in their
 * own dispatch (hipExtLaunchKernel), so their intervals are the kernels'
 * execution times; the other kinds are bracketed by event records on the
 * plan's stream. */
int flame_timing_begin(flame_plan plan);

/* Stop timing, synchronise the plan's stream and report the summed
 * durations in milliseconds and the counts, per kind: [0] row step kernels,
 * [1] column step kernels, [2] diagnostics and other kernels, [3] graph
 * launches (each covering steps_per_graph steps) and persistent launches
 * (each covering the steps of one flame_step call, up to 1000). Bracketed launches that
 * follow each other share their boundary event, so their intervals include
 * the launch gap. ms4 and counts4 are host arrays of 4 entries. */
int flame_timing_end(flame_plan plan, double* ms4, int64_t* counts4);

/* Points per thread of the step kernels for the flames of grid n1 x n2: each
 * length-N transform is owned by N/pts threads holding pts points, with
 * radix-pts passes (col_pts for the column kernel, row_pts for the row
 * kernel; 8 or 16, default 16; 8 only for lengths up to 8192,
 * FLAME_ERR_UNSUPPORTED_SIZE beyond). pts = 12 selects the 12-point plan (a
 * radix-12 pass, then radix 4 and 2) for transforms of 3/4 of the grid on
 * N/16 threads: col_pts = 12 runs the column transforms of the product grid
 * (it needs flame_set_product_grid enabled, FLAME_ERR_INVALID_ARG
 * otherwise), row_pts = 12 forms the quadratic term on 3 N2/4 phi points
 * instead of N2 (n2 >= 64, FLAME_ERR_UNSUPPORTED_SIZE otherwise); for a
 * product of two box-limited fields that grid is also alias-free, as the
 * theta product grid is. Results agree to rounding, not bit for bit; the
 * choice trades registers per thread for waves per transform. */
int flame_set_points_per_thread(flame_plan plan, int32_t n1, int32_t n2, int32_t col_pts, int32_t row_pts);
int flame_get_points_per_thread(flame_plan plan, int32_t n1, int32_t n2, int32_t* col_pts, int32_t* row_pts);

/* Grid on which flame_step (and its graphs) forms the quadratic term of
 * Eq. (1) for the flames of grid n1 x n2: enable = 0, the N1 x N2 grid of the
 * paper's augmented array (Section 3); enable = 1, a product grid of
 * M1 = 3 N1/4 theta rows (n1 >= 128). The product of two fields truncated to
 * |k1| <= K1 = N1/4 - 1 reaches |k1| <= 2 K1; on M1 >= 3 K1 + 1 rows none of
 * its aliases falls inside |k1| <= K1, so the truncated term, and the step,
 * are the same as on N1 rows up to rounding. It moves 3/4 of the
 * intermediate data and does 3/4 of the row transforms. The column
 * transforms then have length 3 N1/4 (radix-16 passes and a radix-6 pass;
 * col_pts = 8 selects the variant whose forward transform runs on twice the
 * threads with 8 points each and whose Wp and Wm transforms run side by
 * side). Diagnostics,
 * state I/O, synthesis and the adjoint always use the N1 x N2 grid. Default:
 * enabled for n1 >= 128. Disabling it while col_pts = 12 fails with
 * FLAME_ERR_INVALID_ARG. Changing it synchronises the stream. */
int flame_set_product_grid(flame_plan plan, int32_t n1, int32_t n2, int32_t enable);
int flame_get_product_grid(flame_plan plan, int32_t n1, int32_t n2, int32_t* enabled);

/* Store kind of the step's intermediates for the flames of grid n1 x n2:
 * enable = 1 makes the row kernel write Q, and the column kernel write Wp and
 * Wm, with non-temporal stores (the lines are not kept in L2 for reuse);
 * enable = 2 makes only Wp and Wm non-temporal, enable = 3 only Q; 0, the
 * default, uses plain stores (other values: FLAME_ERR_INVALID_ARG). The
 * getter returns the same code. The arithmetic and the results are the same
 * either way, bit for bit. A workgroup writes pieces of half a 128-byte line
 * of W (and at some grids of Q); non-temporal pieces are written back
 * without being merged with the other half, so each non-temporal buffer
 * moves more HBM bytes than its plain stores would. Non-temporal stores shorten the kernel that writes
 * and lengthen the one that reads next, which then misses in the caches more
 * often; which way the step gains depends on the grid and on what runs beside
 * it, so flame_autotune measures both. The state, the diagnostics and the
 * adjoint use plain stores. Errors: FLAME_ERR_INVALID_ARG if no flame of the
 * plan has that grid (or a null output pointer). Setting discards the step
 * graph (it is rebuilt at the next graph step). */
int flame_set_streaming_stores(flame_plan plan, int32_t n1, int32_t n2, int32_t enable);
int flame_get_streaming_stores(flame_plan plan, int32_t n1, int32_t n2, int32_t* enabled);

/* Choose the step kernels of each grid group by timing. For every group of
 * equal grids, each configuration runs one untimed and `steps` timed steps of
 * that group (HIP events on the plan's stream), in three rounds over all
 * configurations (the fastest time counts), and the fastest is kept if
 * it runs in at most 98 % of the default's time (16 points per thread, on
 * the product grid where n1 >= 128, plain stores), else the default, so that
 * choices within timing noise of each other do not change from run to run.
 * The configurations are (col_pts, row_pts) in {16, 8} x {16, 8, 12} on the
 * N1-row grid and, for n1 >= 128, {16, 8, 12}^2 on the product grid (row_pts
 * 12 only where n2 >= 64), each with plain and with non-temporal stores
 * (flame_set_streaming_stores). If a group's choice has both Q and W
 * non-temporal, the same kernels with only W and with only Q non-temporal are
 * timed as well, and the faster of the two replaces it if it runs in at most
 * 1/0.98 of its time (it moves fewer bytes). When graphs are in use
 * (flame_set_graph_steps > 0) and the plan has several groups, whose chains
 * run concurrently in a replay, the choices are then refined jointly:
 * coordinate descent over the groups, each trial running `steps` steps of
 * every group at once on streams of their own, a change kept only if it runs
 * in at most 98 % of the best time so far. The states
 * and the step index are saved in the workspace and restored afterwards,
 * also when a trial fails, so the call does not change the simulation; it
 * synchronises the stream. With the persistent launch enabled
 * (flame_set_persistent), whose kernels are fixed, it fails with
 * FLAME_ERR_INVALID_ARG.
 * *n_configs_tried (nullable) receives the number of timed configurations. */
int flame_autotune(flame_plan plan, int32_t steps, int32_t* n_configs_tried);

/* Run flame_step in graphs of `steps` steps (0: direct launches, the default).
 * The graph holds, for every group of flames with equal grids (and equal
 * integrators), the chain row kernel -> column kernel for each step (twice
 * per step for integrating-factor Heun); chains of different groups have
 * no edges between them, so a mixed ensemble runs its groups concurrently.
 * flame_step(n) launches floor(n / steps) graphs and the remainder directly.
 * The graph is built on first use and replayed; the step index is read from
 * the workspace, set by a one-thread kernel before each replay. Calls that
 * discard the graph (a new graph length, points per thread, grid or forcing
 * group) first wait for the plan's stream. */
int flame_set_graph_steps(flame_plan plan, int32_t steps);

/* Run flame_step as one persistent launch (enable = 1) instead of per-group
 * kernels or graphs: a cooperative launch of one co-resident grid whose
 * workgroups step every flame of the plan for up to 1000 steps per launch.
 * Each workgroup runs the step kernels' work (Section 3's two transform
 * passes with the Eq. (1) update between them) on its share of the flames:
 * several small flames alone, or a part of a large flame's row-pair groups
 * and column tiles, meeting that flame's other workgroups at a device-memory
 * counter after each pass. The arithmetic is that of the per-group kernels,
 * so the results are the same bit for bit. Shares are sized so that every
 * workgroup has about the same number of tiles per step.
 *
 * workgroups: the grid size (0: every workgroup that fits on the device,
 * two per compute unit). wait_limit_us: the bound of each wait at a counter,
 * in microseconds (0: 2 s); a wait that runs out makes every workgroup stop,
 * and flame_step returns FLAME_ERR_TIMEOUT with the states undefined. In
 * this mode flame_step waits for the plan's stream before it returns (to
 * read that status). With flame_set_graph_steps(k), 0 < k <= 1000, the
 * launches are replays of a hipGraph holding k steps: a node that zeroes the
 * counters, then the persistent kernel as a cooperative kernel node that
 * reads the step index from the workspace; remaining steps run as direct
 * cooperative launches.
 *
 * Requires every group of the plan on the product grid with col_pts = 12,
 * row_pts = 16, plain stores, integrator 0 and no forcing, with n1 in
 * [128, 1024] and n2 in [128, 2048] (FLAME_ERR_INVALID_ARG otherwise, also
 * from flame_step if a later call changes a group's configuration), and a
 * device with cooperative launches (FLAME_ERR_UNSUPPORTED_SIZE). enable = 0
 * returns to the per-group launches. */
int flame_set_persistent(flame_plan plan, int32_t enable, int32_t workgroups, int32_t wait_limit_us);
/* *enabled: whether flame_step runs persistent launches; *workgroups: the
 * grid of the last one (0 before the first). */
int flame_get_persistent(flame_plan plan, int32_t* enabled, int32_t* workgroups);

/* Release the plan's host metadata (device buffers stay the caller's), after
 * waiting for the plan's stream. */
int flame_destroy(flame_plan plan);

/* Circular (two-dimensional) flames. Section 2 compares the spherical flames
 * with circular ones but gives only Eq. (1); the library takes for them the
 * one-dimensional form of Eq. (1), i.e. Eq. (1) on the modes k1 = 0 (a set
 * the equation maps into itself), for the perturbation Phi(phi, t) of a
 * circle of radius r0(t) = t:
 *   dPhi~_k/dt = (-kappa_k^2/r0^2 + gamma |kappa_k|/(2 r0)) Phi~_k
 *                - 1/(2 r0^2) sum_l kappa_l kappa_{k-l} Phi~_l Phi~_{k-l},
 * kappa_k = seg k, truncated to |k| <= K = n/4 - 1 and evaluated on n points
 * (the augmented-array rule of Section 3), stepped by integrating-factor
 * Euler with Im Phi~_0 = 0 after each step, like flame_step.
 *
 * State of one circle: complex64 spec[k], k = 0 .. K (n/4 entries; the k < 0
 * half follows from Phi~(-k) = conj(Phi~(k)); Im spec[0] must be 0). A batch
 * is n_circles such arrays back to back (dev, caller-owned). The calls need
 * no plan and no workspace: every circle's spectrum stays in registers
 * during a launch, and the twiddles are computed on the device. */
typedef struct {
  int32_t n;        /* points per circle: a power of two in [16, 16384] */
  double gamma;     /* density contrast, >= 0 */
  double seg;       /* segment integer (1: the whole circle), > 0 */
  double t0;        /* time of step index 0, > 0 */
  double dt;        /* time step, > 0 */
} flame_circle_desc;

/* Bytes of one circle's state (n/4 complex64). */
int flame_circle_state_bytes(const flame_circle_desc* desc, size_t* bytes);

/* Advance every circle of the batch `states` (dev, n_circles states, 8-byte
 * aligned) from step index n (time t0 + n dt) by nsteps >= 0 steps, in
 * place, on hip_stream. Circles 2c and 2c + 1 are stepped as a pair that
 * shares one complex transform: results do not depend on the batch's size or
 * order beyond rounding, and are reproducible bit for bit for a fixed batch,
 * but a circle whose state turns non-finite also spoils its partner. */
int flame_circle_step(const flame_circle_desc* desc, int32_t n_circles, void* states, int64_t n, int32_t nsteps,
                      void* hip_stream);

/* Averages of each circle at step index n, in double (dev out4, 4 doubles
 * per circle): [0] mean radius r0 + Re Phi~_0, [1] averaged velocity
 * <Phi_t> = dPhi~_0/dt = sum_k w_k kappa_k^2 |Phi~_k|^2 / (2 r0^2) (w = 1 at
 * k = 0, 2 elsewhere), [2] length excess: the grid mean of sqrt(1 + x) - 1,
 * x = Phi_phi^2 / r0^2 (kappa scaling), as x / (1 + sqrt(1 + x)), [3] 1 if
 * every stored coefficient is finite, else 0 (non-finite coefficients enter
 * the averages as zero, so that they do not reach the partner circle's). */
int flame_circle_diagnostics(const flame_circle_desc* desc, int32_t n_circles, const void* states, int64_t n,
                             double* out4, void* hip_stream);

/* Allocation-free stepping, for callers that cannot allocate device memory
 * or build a plan (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Advances one flame described by `desc`
 * (host) by nsteps >= 0 integrating-factor Euler steps of Eq. (1), with
 * the kernel sequence flame_step runs on a fresh plan in its default
 * configuration (product grid for n1 >= 128, 16 points per thread, plain
 * stores, direct launches): the column transforms of the state, then a row
 * and a column kernel per step. `state` (dev, flame_state_bytes, 16-byte
 * aligned, the state layout above) holds the state at step index n
 * (time t0 + n dt) and is updated in place; the work is queued on
 * hip_stream (a hipStream_t, 0 for the null stream) of the current device.
 * Only r0_law = 0 and integrator = 0 are accepted (FLAME_ERR_INVALID_ARG
 * otherwise).
 *
 * The workspace (the intermediates W and Q, the twiddle tables, the flame
 * descriptor) is a static device array of FLAME_NOALLOC_SCRATCH_BYTES that
 * the library holds on every GPU it runs on until the process ends; the call
 * allocates nothing. A grid whose workspace exceeds it (2048 x 4096 fits)
 * fails with FLAME_ERR_WORKSPACE_TOO_SMALL before anything is queued. Every
 * call on one GPU shares that GPU's array and overwrites it: calls that
 * overlap on one GPU (other streams or host threads) race, while calls
 * queued in order on one stream do not. Nothing in the array needs to start
 * at zero: each call writes every location that a kernel reads for a stored
 * result. */
#define FLAME_NOALLOC_SCRATCH_BYTES (48u * 1024u * 1024u)
int flame_step_noalloc(const flame_desc* desc, void* state, int64_t n, int32_t nsteps, void* hip_stream);

/* Text of the last error raised on the calling thread ("" if none). */
const char* flame_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FLAME_H */
