/*
 * wt.h -- time-dependent weighting field H(x,t) of a 3D diamond pixel with
 * resistive graphitised columns, and the induced current of drifting charge
 * carriers (extended Ramo-Shockley theorem, Eq. 1 of the paper), on one
 * AMD Instinct MI355X (gfx950).
 *
 * Two calls carry the method (paper, Section 2 "workflow of micro-steps":
 * geometry -> correlation function H(x,t); H + carrier paths -> currents):
 *
 *   wt_h_solve  geometry + column resistivities + frequency/time grid -> H
 *               (abstract and Section 3: point charges on the electrode
 *               boundaries fitted to the boundary conditions, i.e. the
 *               fundamental solutions, then a spectral extension to the bulk;
 *               the equation solved is the quasi-static, third-order limit of
 *               Maxwell's equations, div((sigma + i w eps) grad psi) = 0 per
 *               frequency, followed by a frequency-to-time transform)
 *   wt_current  H + carrier polylines -> i_track(t)   (Eq. 1, introduction;
 *               Section 3: the convolution of every carrier's velocity with H)
 *
 * and wt_h_gradient gives dL/d(column resistivities, radii) of a loss of the
 * currents by the adjoint of both calls.
 *
 * Conventions shared by every call:
 *  - SI units (m, s, ohm*m, C, V).  V_w = 1 V.
 *  - All device buffers are caller-owned (e.g. torch tensors); the library
 *    never allocates, frees or retains device memory.  Pointers prefixed d_
 *    are device pointers; everything else is host memory read during the
 *    call only.
 *  - Work is enqueued on the context's HIP stream and returns without
 *    waiting, except where a call says it synchronises.
 *  - Every function returns wt_status (0 = WT_OK, negative = error).  No
 *    exception or abort crosses this boundary.  On WT_E_HIP the runtime's
 *    message is kept in the context (wt_context_last_error).
 *  - A context is not thread-safe; a plan is immutable and may be shared,
 *    except while wt_h_plan_tune changes it.
 */
#ifndef WT_H
#define WT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    WT_OK = 0,
    WT_E_INVALID_ARG = -1,      /* null pointer, non-positive or non-finite size/value */
    WT_E_GEOMETRY = -2,         /* column off a grid node, overlapping columns,
                                   column outside the cell, radius too large */
    WT_E_UNSUPPORTED_SIZE = -3, /* grid size odd or not 2*3*5-smooth, or beyond a
                                   limit listed below */
    WT_E_WORKSPACE = -4,        /* a caller buffer is smaller than required */
    WT_E_SINGULAR = -5,         /* zero pivot in a collocation solve */
    WT_E_NOT_CONVERGED = -6,    /* refinement did not reach ir_tol */
    WT_E_HIP = -7               /* HIP runtime error (message in the context) */
} wt_status;

typedef enum {
    WT_F64 = 0,   /* bulk FFTs, H and the convolution in double */
    WT_F32 = 1    /* bulk FFTs, H and the convolution in float (the boundary
                     fit and the time transform stay in double) */
} wt_precision;

/* Periodic cell L_x x L_y x L_z on an N_x x N_y x N_z grid of nodes
 * (i h_x, j h_y, k h_z), h_a = L_a / N_a.  N_a even, 2*3*5-smooth, 4..1024.
 * The diamond bulk has relative permittivity eps_r; sigma_bulk must be 0. */
typedef struct {
    double Lx, Ly, Lz;
    int Nx, Ny, Nz;
    double eps_r;
    double sigma_bulk;
} wt_cell;

/* A resistive column: axis (x, y) on a grid node, radius, contact end
 * z_contact (held at v_applied) and free end z_free, both in [0, L_z].
 * n_colloc >= 2 nodes z_m = z_contact + m (z_free - z_contact)/(n_colloc-1).
 * resistivity[0..n_resistivity-1] (ohm*m, > 0) are quarter-columns in
 * parallel; the column conductivity is the mean of 1/resistivity. */
typedef struct {
    double x, y;
    double radius;
    double z_contact, z_free;
    double resistivity[4];
    int n_resistivity;
    int n_colloc;
    double v_applied;
} wt_column;

/* Frequencies f_j = j df (j < n_freq), times t_n = n dt (n < n_time).
 * n_freq 1..65535; n_time 1..512. */
typedef struct {
    int n_freq;
    double df;
    int n_time;
    double dt;
} wt_spectrum;

typedef enum {
    WT_H_PLAIN = 0,        /* H stored in the path's precision (double or float) */
    WT_H_F16_SCALED = 1    /* H stored as float16 values of H * h_scale, with
                              h_scale = 2^s chosen from a bound on |H| so that
                              every stored magnitude is <= 16384 (requires
                              WT_F32 and a grid the register-FFT synthesis
                              takes: N_z in {64, 128, 256, 512} with at most 4
                              columns, or two columns and an even 2,3,5-smooth
                              N_z in [72, 320]: 72, 80, 90, 96, 100, 108, 120,
                              144, 150, 160, 162, 180, 192, 200, 216, 240, 250,
                              270, 288, 300, 320); the synthesis and the
                              convolution compute in float */
} wt_h_format;

typedef struct {
    int precision;      /* wt_precision */
    int ir_max_iter;    /* refinement sweeps after the LU solve, 0..16 */
    double ir_tol;      /* target normwise backward error (>= 0) */
    int h_format;       /* wt_h_format */
    int fft_schedule;   /* register-FFT synthesis: which of the size's
                           compiled schedules (factor pair and staging block)
                           to start from, 0 .. wt_fft_schedule_count(N_z) - 1
                           (0: the default, the fastest measured; in double
                           only those that fit in LDS count); must be 0 for
                           grids without a register form (WT_E_INVALID_ARG
                           otherwise) */
} wt_h_options;

/* Number of register-FFT synthesis schedules (a factor pair N_z = N1 x N2
 * and a staging block of 8 or 16 samples) compiled for a float plan with
 * two columns and this N_z: 2 for 64, 128 and 256 (blocks of 8 and 16), 1
 * for 512; 3 for each non-power-of-two size listed at WT_H_F16_SCALED; 0
 * otherwise. */
int wt_fft_schedule_count(int n_z);

/* Filled by wt_h_solve when a report pointer is given (that call then
 * synchronises the stream). */
typedef struct {
    double backward_error_max;  /* max over frequencies, normwise, after refinement */
    double pivot_ratio_max;     /* max over frequencies of max|U_ii| / min|U_ii| */
    int ir_iters_max;           /* refinement sweeps used (max over frequencies) */
    int singular_count;         /* frequencies whose LU met a zero pivot */
    double h_scale;             /* stored value = H * h_scale (1 for WT_H_PLAIN) */
} wt_h_report;

/* Sizes and byte offsets of a plan.  H is stored time-blocked:
 *   H[x][y][tb][z][tin][a],  t = tb * h_time_block + tin,  a = component x,y,z
 * where the last block holds n_time - tb*h_time_block samples; for node
 * (x, y, z), time t and component a the element index is
 *   (x*Ny + y)*Nz*n_time*3 + tb*h_time_block*Nz*3 + z*Tb*3 + tin*3 + a
 * with Tb the length of block tb.  Each node's lag series is contiguous
 * within a block.  The element type is double (WT_F64), float (WT_F32) or,
 * for WT_H_F16_SCALED, float16 holding H * h_scale; the buffer then ends
 * with a float 1 / h_scale at byte offset h_decode_offset (written by
 * wt_h_solve, read by wt_current), so that H carries its own scale.
 * The workspace offsets locate intermediate results (for inspection):
 *   A      double  [n_q][n_q]        collocation matrix, V/C
 *   qw     double2 [n_freq][n_q+1]   charges q(w_j) (C/V) then the gauge c
 *   qt     double  [n_time][n_q]     charges q(t_n), C/(V s)
 *   qhat   T2      [n_time][n_cols][Nz/2]  per-column z-transform of q(t_n)
 *   ehat   T2      [Nx][Ny][Nz/2][3] in-plane field table of one unit column */
typedef struct {
    size_t workspace_bytes;
    size_t h_bytes;
    int h_time_block;
    int n_q;
    size_t off_A, off_qw, off_qt, off_qhat, off_ehat;
    int h_format;               /* wt_h_format of the plan */
    size_t h_decode_offset;     /* WT_H_F16_SCALED: byte offset of 1/h_scale in H; else 0 */
} wt_h_layout;

typedef struct wt_context wt_context;
typedef struct wt_h_plan wt_h_plan;

/* Carriers for wt_current.  Element type of d_pos, d_charge and the output
 * follows the plan's precision (double or float).
 *   d_pos    [n_carriers][n_time+1][3]  polyline P_c(t_0..t_n_time), m, any
 *            real coordinates (the cell is periodic)
 *   d_charge [n_carriers]  carrier charge, C
 *   d_track  [n_carriers]  track index in [0, n_tracks); carriers outside
 *            this range are skipped */
typedef struct {
    int n_carriers;
    int n_tracks;
    const void* d_pos;
    const void* d_charge;
    const int* d_track;
} wt_carriers;

/* Create a context bound to HIP device `hip_device` and the HIP stream
 * `hip_stream` (a hipStream_t; NULL = the default stream).  Fails with
 * WT_E_HIP when no such device exists or the runtime cannot reach it.  The
 * library calls the HIP runtime it was loaded with: device memory and the
 * stream must belong to that same runtime (one HIP runtime per process). */
wt_status wt_context_create(wt_context** ctx, int hip_device, void* hip_stream);
wt_status wt_context_destroy(wt_context* ctx);
/* Last HIP error message of the context ("" if none); owned by the context.
 * With ctx = NULL: the message of this thread's last failed
 * wt_context_create, owned by the library. */
const char* wt_context_last_error(const wt_context* ctx);

/* Per-stage timing (HIP events on the context's stream).  When enabled,
 * every wt_h_solve / wt_current records an event between its stages;
 * wt_context_stage_times synchronises the stream and returns the stage
 * durations of the last call, in milliseconds, with their names
 * (wt_stage_name).  n_out receives the number of stages written. */
wt_status wt_context_enable_timing(wt_context* ctx, int enable);
wt_status wt_context_stage_times(wt_context* ctx, double* ms, int max_stages, int* stage_ids, int* n_out);
const char* wt_stage_name(int stage_id);

/* Validate a problem and build a plan (host only, no GPU work).  The plan
 * copies everything it needs.  layout receives the required workspace and H
 * sizes. */
wt_status wt_h_plan_create(const wt_cell* cell, const wt_column* cols, int n_cols,
                           const wt_spectrum* spectrum, const wt_h_options* options,
                           wt_h_plan** plan, wt_h_layout* layout);
wt_status wt_h_plan_destroy(wt_h_plan* plan);
wt_status wt_h_plan_layout(const wt_h_plan* plan, wt_h_layout* layout);

/* Result of wt_h_plan_tune. */
typedef struct {
    int n_candidates;    /* launch configurations timed (1: nothing to tune) */
    int h_time_block;    /* the chosen time block of the H layout */
    int threads;         /* workgroup size of the chosen synthesis launch */
    double ms_chosen;    /* synthesis time of the chosen configuration (-1 if none timed) */
    double ms_default;   /* the plan's configuration before tuning (-1 if none timed) */
    int fft_n1;          /* register-FFT synthesis: N_z = fft_n1 x (N_z / fft_n1)
                            (pass-1 lanes per transform); 0: the LDS Stockham
                            synthesis */
    int from_cache;      /* 1: the choice came from the context's tuning cache
                            (nothing timed; ms_chosen is the cached time) */
} wt_tune_report;

/* Tuning cache of the context (a text file): wt_h_plan_tune first looks up
 * the plan's device (architecture, compute units) and grid (N_x, N_y, N_z,
 * n_time, precision, h_format, n_cols) there and applies a cached choice
 * that is still among its candidates without timing; otherwise it times the
 * candidates as usual and rewrites the file with the new entry.  The file is
 * read here (a missing file is an empty cache; a malformed one gives
 * WT_E_INVALID_ARG and leaves the cache off); path NULL or "" turns the
 * cache off.  One context per file: concurrent writers are not coordinated. */
wt_status wt_context_set_tune_cache(wt_context* ctx, const char* path);

/* Autotuning of the synthesis launch for this plan's grid on this device:
 * runs wt_h_solve once, then times every candidate configuration of the LDS
 * Stockham synthesis (used where the register-FFT synthesis has no form: N_z
 * neither in {64, 128, 256, 512} nor among the smooth sizes listed at
 * WT_H_F16_SCALED; a smooth size in double or without exactly two columns;
 * N_z = 512 in double; more than 4 columns): its time
 * block (powers of two up to 32 whose staging fits in LDS) and workgroup
 * size (256, 512), or of the register-FFT synthesis: the size's schedules
 * (factor pairs N_z = N1 x N2 and staging blocks of 8 or 16 samples)
 * compiled into the library; two launches each after a warm-up,
 * keeps the fastest in the plan and rewrites H in that configuration.  The
 * register-FFT synthesis of a power of two has two schedules (blocks of 8
 * and 16 samples), one at N_z = 512 (n_candidates = 1).  This call changes the
 * plan: the layout's h_time_block may differ afterwards (re-read it with
 * wt_h_plan_layout; h_bytes and the workspace size do not change), so no
 * other call may use the plan concurrently.  Synchronises the stream.
 * report may be NULL. */
wt_status wt_h_plan_tune(wt_context* ctx, wt_h_plan* plan, void* d_workspace, size_t workspace_bytes,
                         void* d_h, size_t h_bytes, wt_tune_report* report);

/* Solve for H: Green's tables and collocation matrix, one bordered complex
 * FP64 collocation solve (LU with partial pivoting + refinement) per
 * frequency, time transform of the charges, in-plane field table, and the
 * per-column synthesis of H(x, y, z, t) for every grid node and time sample.
 * d_workspace: >= layout.workspace_bytes, 256-byte aligned; d_h: >=
 * layout.h_bytes.  With report != NULL the call synchronises, fills the
 * report and returns WT_E_SINGULAR / WT_E_NOT_CONVERGED when they occurred
 * (H is still written).  Without a report these conditions are not checked. */
wt_status wt_h_solve(wt_context* ctx, const wt_h_plan* plan,
                     void* d_workspace, size_t workspace_bytes,
                     void* d_h, size_t h_bytes, wt_h_report* report);

/* Size of the static workspace of wt_h_solve_static, per GPU. */
#define WT_STATIC_WORKSPACE_BYTES ((size_t)32 << 20)

/* wt_h_solve for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  The
 * workspace is a library-owned static device array of
 * WT_STATIC_WORKSPACE_BYTES (32 MiB) on every GPU the library runs on, held
 * until the process ends; nothing is allocated or freed by this call.  The
 * caller still passes H (d_h, >= layout.h_bytes, 16-byte aligned).  Plans
 * whose layout.workspace_bytes exceeds WT_STATIC_WORKSPACE_BYTES are
 * rejected with WT_E_WORKSPACE before any work is enqueued (the message in
 * the context gives both sizes).  Same kernels, results and report as
 * wt_h_solve; the intermediates (collocation matrix, charges, field table)
 * are left in the static workspace, which keeps the last call's contents.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, threads or contexts) race and must be
 * serialised by the caller. */
wt_status wt_h_solve_static(wt_context* ctx, const wt_h_plan* plan, void* d_h, size_t h_bytes,
                            wt_h_report* report);

/* Which form wt_current takes on this context when it is given a workspace:
 * 0 (the default) bins the moving steps from 2^24 polyline steps
 * (n_carriers * n_time) on and gathers per carrier below that, where it is
 * faster; 1 bins at any size; 2 never bins.  Results agree to rounding. */
wt_status wt_context_set_current_form(wt_context* ctx, int form);

/* Bytes of the workspace of wt_current for n_carriers carriers and room for
 * max_events moving steps (max_events <= 0: n_carriers * n_time, every step
 * of every carrier; at most 2^32 - 16 are used).  The fixed part (control
 * words, bin counts and offsets over the grid's cell columns and z-tiles,
 * one 8-byte step mask per carrier and 64 steps) is needed in full; each
 * event then takes 32 bytes (64 for a WT_F64 plan). */
wt_status wt_current_workspace(const wt_h_plan* plan, int n_carriers, long long max_events, size_t* bytes);

/* Induced current (Eq. 1): for every carrier and every polyline step m with a
 * non-zero displacement dx = P(t_{m+1}) - P(t_m), the field at the step
 * midpoint (trilinear interpolation of the nodal H, periodic wrap) at lag
 * n - m is projected on dx and accumulated:
 *   i[track][n] = -(1/V_w) sum_{c in track} q_c sum_{m<=n} H(xbar_{c,m}, t_{n-m}) . dx_{c,m}
 * d_h is H as written by wt_h_solve for the same plan; d_i_out [n_tracks]
 * [n_time] is overwritten.
 * With a workspace (d_workspace 256-byte aligned, at least
 * wt_current_workspace(plan, n_carriers, 1) bytes, overwritten), the moving
 * steps are binned by grid cell and H is read node column by node column,
 * each node's lag series once (the fast form).  If the moving steps exceed
 * the events that fit the workspace, the device falls back to the form
 * without a workspace in the same call (same results, nothing synchronises).
 * d_workspace NULL: one wavefront per carrier gathering its steps' corners.
 * Summation order across carriers is not fixed (atomic accumulation), so
 * results can differ in the last bits.  Outside stream capture the binned
 * form adds its overflow records (tracks past a column's table) on a stream
 * of the context beside the node-column accumulation, forked from and joined
 * back to the context's stream by events; the call stays stream-ordered. */
wt_status wt_current(wt_context* ctx, const wt_h_plan* plan, const void* d_h,
                     const wt_carriers* carriers, void* d_workspace, size_t workspace_bytes,
                     void* d_i_out);

/* One pass of the whole path (Sections 3 and 4): wt_h_solve into d_h, then
 * wt_current (Eq. 1) on that H, with the arguments, checks, results and
 * report of the two calls (the report covers the H solve; with a report the
 * call synchronises).  The current's binning needs only the carriers, so it
 * runs on a stream of the context beside the synthesis: forked from the
 * context's stream by an event after the boundary fit and the field table,
 * joined back by an event before the accumulation.  Under stream capture
 * the two run one after the other on the context's stream.  The stage time
 * "current_binning" is then the wait for the binning after the synthesis.
 * Stream-ordered like every call: the next call on the context's stream
 * sees the current written. */
wt_status wt_step(wt_context* ctx, const wt_h_plan* plan,
                  void* d_workspace, size_t workspace_bytes, void* d_h, size_t h_bytes,
                  const wt_carriers* carriers, void* d_cur_workspace, size_t cur_workspace_bytes,
                  void* d_i_out, wt_h_report* report);

/* Batched forward runs over many geometry variants (each variant is one
 * cell, column set and spectrum: one plan; the workloads of the paper's
 * Section 5 results vary pitch, diameter and resistivity).  For every item,
 * wt_h_solve followed by wt_current, exactly as the two calls would run
 * them; the items are spread over n_lanes HIP streams that fork from the
 * context's stream and join it again, so that one item's small launches
 * (tables, boundary fit, time transform) overlap another's synthesis.
 *   items        [n_items] host array; plan, carriers as for wt_current,
 *                d_current [n_tracks][n_time] in the plan's precision
 *   d_workspace  [n_lanes] device buffers of workspace_bytes each (256-byte
 *                aligned), d_h [n_lanes] buffers of h_bytes each (16-byte
 *                aligned): lane l's scratch, reused by its items in turn
 *   item_status  [n_items] host array or NULL: WT_OK, or why item i was
 *                skipped without running (WT_E_WORKSPACE: its plan's
 *                workspace or H does not fit a lane's buffers;
 *                WT_E_INVALID_ARG: no plan, output or carriers)
 * Items are taken longest first (H bytes plus a fixed per-item cost) and
 * each goes to the lane with the least work so far; a lane runs its items
 * in that order.  n_lanes: 1..8.  Stream-ordered like the other calls:
 * nothing is waited for, so the whole call can be captured into a HIP graph
 * (the lanes join the capture through events); the lanes' streams (default
 * priority, non-blocking) and events are created by the first call on the
 * context, which therefore must not itself be under capture.  Returns WT_OK
 * when every item ran, else the status of the first skipped item
 * (WT_E_INVALID_ARG for bad arguments, with nothing run). */
typedef struct {
    const wt_h_plan* plan;
    wt_carriers carriers;
    void* d_current;
} wt_batch_item;

#define WT_MAX_LANES 8

wt_status wt_batch_run(wt_context* ctx, int n_items, const wt_batch_item* items, int n_lanes,
                       void* const* d_workspace, size_t workspace_bytes,
                       void* const* d_h, size_t h_bytes, int* item_status);

/* Readout electronics and timing features (the workflow's last step,
 * Section 2: the induced signals convolved with the transfer function of the
 * readout electronics, plus noise; the front-end model is the caller's).
 * For every track k and sample n < n_time:
 *   v[k][n] = dt * sum_{m<=n} g[n-m] i[k][m] + noise_sigma * noise[k][n]
 * and features[k] = {A, t_peak, t_cfd}:
 *   n_p = the first index of max_n |v[k][n]|, A = v[k][n_p] (signed);
 *   with u = sign(A) v: t_peak = (n_p + d) dt, d the vertex offset of the
 *     parabola through u[n_p-1], u[n_p], u[n_p+1] (0 at the ends of the
 *     record or where those samples are not concave);
 *   t_cfd = the last upward crossing of cfd_fraction * |A| by u before n_p,
 *     interpolated linearly between samples (NaN if none, or if A = 0).
 * Device arrays: d_current [n_tracks][n_time] (as written by wt_current),
 * d_response [n_time] (the sampled impulse response g, 1/s), d_noise
 * [n_tracks][n_time] (e.g. standard normal samples; NULL for none),
 * d_signal [n_tracks][n_time] and d_features [n_tracks][3] (overwritten).
 * Element type double (WT_F64) or float (WT_F32).  n_tracks >= 1, n_time
 * 1..512, dt > 0, noise_sigma >= 0, 0 < cfd_fraction < 1; otherwise
 * WT_E_INVALID_ARG (n_time > 512: WT_E_UNSUPPORTED_SIZE). */
wt_status wt_electronics(wt_context* ctx, int precision, int n_tracks, int n_time, double dt,
                         const void* d_current, const void* d_response, const void* d_noise, double noise_sigma,
                         double cfd_fraction, void* d_signal, void* d_features);

/* Bytes of the gradient workspace of wt_h_gradient for a plan and n_tracks
 * tracks (WT_E_UNSUPPORTED_SIZE when the plan has more than 128 charges). */
wt_status wt_h_gradient_workspace(const wt_h_plan* plan, int n_tracks, size_t* bytes);

/* Gradient of a loss L of the currents with respect to every column's
 * quarter-column resistivities and radius and to the pixel pitch (the
 * electrode parameters of the paper's Section 5 results: resistance
 * R = 4 rho L / (pi d^2) through the resistivity and the diameter, and the
 * pixel geometry), by the adjoint of the whole path.
 *   d_grad_current [n_tracks][n_time]: dL/di, element type of the plan's
 *     precision;
 *   d_grad_params  [n_cols*5 + 1] double (overwritten): for column w,
 *     [5w + p] = dL/d resistivity[p] (ohm*m) for p < n_resistivity (0 in the
 *     unused slots) and [5w + 4] = dL/d radius (m); then [5 n_cols] =
 *     dL/d pitch (m): the derivative under a uniform scaling of the in-plane
 *     cell size L_x, L_y, the column axes and the carriers' in-plane
 *     coordinates (the grid counts, radii and z extents held), per metre of
 *     L_x.
 * The carriers are those given to wt_current.  For the resistivities and
 * radii their polylines are held fixed; for the pitch their in-plane
 * coordinates scale with the cell (trilinear weights unchanged).
 * d_workspace must hold what wt_h_solve wrote for this plan (the collocation
 * matrix, the charges q(w) of every frequency and the field table); it is
 * only read.  H itself is not needed: the adjoint projects every moving step
 * of the carriers on the column spectra, correlates with dL/di over the lags,
 * transposes the z-transform and the time quadrature, solves the transposed
 * boundary-fit system S(w)^T lambda = dL/dq(w) at every frequency (FP64,
 * LU with partial pivoting and refinement) and contracts lambda with
 * dS/dtheta: the RC-line block through the column conductivity and radius,
 * the collocation matrix through the collocation offset r and the source
 * width r/4 (and the cell size for the pitch).  For the pitch the current also
 * changes at fixed charges, through the field table and the in-plane
 * displacements: a second projection of the moving steps, with the pitch
 * derivative of the field table, is taken against the column spectra.
 * d_grad_workspace: >= wt_h_gradient_workspace bytes, 256-byte aligned,
 * overwritten.  Plans with more than 128 charges: WT_E_UNSUPPORTED_SIZE.
 * With report != NULL the call synchronises and reports the transposed
 * solves (WT_E_SINGULAR / WT_E_NOT_CONVERGED as for wt_h_solve; h_scale 1). */
wt_status wt_h_gradient(wt_context* ctx, const wt_h_plan* plan,
                        const void* d_workspace, size_t workspace_bytes,
                        const wt_carriers* carriers, const void* d_grad_current,
                        void* d_grad_workspace, size_t grad_workspace_bytes,
                        double* d_grad_params, wt_h_report* report);

const char* wt_status_string(wt_status status);

#ifdef __cplusplus
}
#endif

#endif /* WT_H */
