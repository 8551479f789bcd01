// Internal definitions shared by the HIP sources of the library (not part of
// the C ABI).  Complex arithmetic, the validated plan, and the kernel
// launchers that the ABI layer calls.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace wt {

constexpr double kEps0 = 8.8541878128e-12;   // vacuum permittivity, F/m (CODATA 2018)
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxCols = 8;
constexpr int kMaxRadices = 16;
constexpr int kMaxTime = 512;
constexpr double kCutoffExponent = 40.0;       // converged Green's sum: k^2 s^2 / 2 <= 40
constexpr double kColWidthFraction = 0.25;     // boundary-fit source width = radius / 4

template <typename T>
struct cplx {
    T re, im;
};

template <typename T>
__host__ __device__ inline cplx<T> mk(T r, T i) { return cplx<T>{r, i}; }
template <typename T>
__host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ inline cplx<T> scale(cplx<T> a, T s) { return {a.re * s, a.im * s}; }
template <typename T>
__host__ __device__ inline cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T>
__host__ __device__ inline cplx<T> mul_i(cplx<T> a) { return {-a.im, a.re}; }   // i * a

struct Column {
    double x, y, radius, z_contact, z_free;
    double sigma;        // mean conductivity of the quarter-columns, S/m
    double resistivity[4];   // the quarter-columns' resistivities, ohm m
    int n_res;
    double v_applied;
    int n;               // nodes
    int ix, iy;          // axis grid node
    int offset;          // first unknown of this column
    double width;        // boundary-fit source width
    int mmax[3];         // converged mode box |m_a| <= mmax[a]
};

struct Plan {
    double L[3];
    int N[3];
    double eps;            // eps_r * eps0
    int n_cols;
    Column col[kMaxCols];
    int n_q;               // source charges
    int n;                 // n_q + 1 (gauge)
    int n_freq, n_time;
    double df, dt;
    int last_weight_one;   // last frequency is the Nyquist frequency 1/(2 dt)
    int precision;         // 0 double, 1 float
    int h_format;          // 0 H in the path's precision, 1 float16 holding H * h_scale
    int ir_max_iter;
    double ir_tol;
    double s_bulk[3];
    int nkz_tab;           // k_z >= 0 entries per Green's table row (max over columns)
    int tb;                // time block of the H layout
    int synth_kernel;      // 2: pipelined register FFTs, 0: LDS Stockham
    int synth_threads;     // workgroup size of the LDS Stockham synthesis (256, 512 or 1024)
    int synth_n1;          // register FFTs: N_z = synth_n1 x (N_z / synth_n1)
    int synth_tbc;         // register FFTs: samples per staged block (16 or 8)
    int nzh;               // Nz / 2
    int nrad[3];
    int rad[3][kMaxRadices];
    // workspace layout (bytes)
    size_t off_tw[3], off_g, off_A, off_lu, off_piv, off_qw, off_rep, off_qt, off_qhat, off_ehat;
    size_t off_hscale;     // float16 H: [0] float h_scale, [64 B on] uint32 max |Ehat| per k_z, then float qsum per k_z
    size_t ws_bytes, h_bytes;
    size_t h_values_bytes; // bytes of the values of H; for float16 H the float 1/h_scale follows
};

// Buffers of the adjoint (gradient) computation, byte offsets into the
// caller's gradient workspace.
struct GradLayout {
    int n_tracks;
    size_t off_phi;      // [n_tracks][n_time][n_cols][nzh] complex, path precision: event projections
    size_t off_phis;     // the same for the pitch derivative of the current at fixed charges
    size_t off_gamma;    // [n_time][n_cols][nzh] complex double: dL/d(column spectra)
    size_t off_gammas;   // the same lag correlation of the pitch projections
    size_t off_eds;      // [N_x][N_y][nzh][3] complex, path precision: pitch derivative of the field table
    size_t off_pitch;    // [n_time] double: per-lag terms of the pitch derivative at fixed charges
    size_t off_gbar;     // [n_time][n_q] double: dL/dq(t)
    size_t off_rhs;      // [n_freq][n] complex double: right-hand sides of the transposed solves
    size_t off_lam;      // [n_freq][n] complex double: adjoint charges
    size_t off_rep;      // [n_freq] SolveReport of the transposed solves
    size_t off_part;     // [n_freq][n_cols][2] double: per-frequency RC-line terms
    size_t off_K;        // [n_q][n_q] double: sum over frequencies of Re(lambda_i q_j)
    size_t off_gd;       // [3][n_cols][n_cols][nkz_tab] double: lattice-sum derivatives
    size_t off_prod;     // [3][n_q][n_q] double: collocation-matrix derivative terms
    size_t bytes;
};

// Per-frequency solve diagnostics written by the solve kernel.
struct SolveReport {
    double backward_error;
    double pivot_ratio;
    int iters;
    int singular;
};

// Kernel launchers (each returns the HIP error of its launch).
hipError_t launch_twiddles(const Plan& p, void* ws, hipStream_t s);
hipError_t launch_green_tables(const Plan& p, void* ws, hipStream_t s);
hipError_t launch_collocation_solve(const Plan& p, void* ws, hipStream_t s);
hipError_t launch_time_transform(const Plan& p, void* ws, hipStream_t s);
hipError_t launch_field_table(const Plan& p, void* ws, hipStream_t s);
hipError_t launch_h_scale(const Plan& p, void* ws, void* h, hipStream_t s);
hipError_t launch_synthesis(const Plan& p, void* ws, void* h, hipStream_t s);
hipError_t launch_electronics(int precision, int n_tracks, int nt, double dt, const void* cur, const void* g,
                              const void* noise, double sigma, double frac, void* v, void* feat, hipStream_t s);
// Shape of the binned convolution (k_conv.hip).  Events are counted per grid
// cell and written as four node-column records each (one per (x, y) corner
// column of the cell), ordered by (node column, lower z-node).  One workgroup
// per node column, one lane per output sample: threads = 64 ceil(n_time /
// 64); the column's z-nodes are taken zt at a time.  LDS: the tile's zt + 1
// nodes as rows of 64 + threads lags (4 values each, of the stored H type),
// and the column's record offsets per z-node (N_z + 1).  Records are read
// from global memory into scalar registers.  Per-track sums live in
// registers: slots of them (the column's track table).
struct ConvTiling {
    int threads, n_chunks;
    int zt;
    int slots;
    int rl;               // lags per LDS row: 64 zero lags, n_time rounded up to 16
    int lb;               // bytes per lag in a row (4 values of the stored H type)
    size_t n_cells, n_cols;
    size_t off_zoff, lds_bytes;
};
// per-track sums per lane (registers), float and double path; the last
// one takes the tracks past the column's table.  16 leaves each lane 72
// registers, so that four workgroups of 448 lanes share a CU; the table
// holds the tracks with the most records (at 256x256x512, 1e6 carriers of
// 100 tracks, 0.5% of the records belong to tracks past it).
constexpr int kConvSlotsF32 = 16;
constexpr int kConvSlotsF64 = 16;
// z-nodes per tile for h_elem bytes per stored value: at 400 samples the
// rows take 33 KB (float16: four workgroups per CU) or 45 KB (float, double:
// three), and (zt + 1) nodes' lags are in flight per lane in registers
__host__ __device__ constexpr int conv_tile_nodes(int h_elem) { return h_elem == 2 ? 8 : (h_elem == 4 ? 5 : 2); }
inline ConvTiling conv_tiling(const Plan& p) {
    ConvTiling t{};
    auto a16 = [](size_t v) { return (v + 15) & ~(size_t)15; };
    const int nw = (p.n_time + 63) / 64;
    t.threads = 64 * nw;
    t.n_chunks = nw;
    const int h_elem = p.precision == 0 ? 8 : (p.h_format == 1 ? 2 : 4);
    t.zt = conv_tile_nodes(h_elem);
    t.slots = (p.precision == 0 ? kConvSlotsF64 : kConvSlotsF32) - 1;
    // rows of 64 + n_time lags (rounded up to 16); lanes past the last
    // sample read up to threads - n_time lags further, which stay inside the
    // allocation (garbage they drop)
    t.rl = 64 + ((p.n_time + 15) & ~15);
    t.lb = 4 * h_elem;
    const size_t rows = (size_t)(t.zt + 1) * t.rl * 4 * h_elem + (size_t)64 * 4 * h_elem;
    t.off_zoff = a16(rows);
    t.lds_bytes = t.off_zoff + a16((size_t)(p.N[2] + 1) * sizeof(unsigned));
    t.n_cols = (size_t)p.N[0] * p.N[1];
    t.n_cells = t.n_cols * p.N[2];
    return t;
}
// Workspace of the binned convolution (byte offsets): control words, cell
// counts and fill counters (zeroed together), record offsets per (node
// column, z-node) (n_cells + 1), scan block sums, per cell the first record
// of its events in each of its four bins (4 u32), the per-(carrier, 64
// steps) moving masks, the per-column track tables, then the records (as
// many as fit; four per event).
struct CurrentLayout {
    size_t off_ctl, off_count, off_fill, off_offs, off_bsum, off_base, off_mask, off_tables, off_records, fixed_bytes;
};
inline CurrentLayout current_layout(const Plan& p, const ConvTiling& t, long long n_carriers) {
    auto a256 = [](size_t v) { return (v + 255) & ~(size_t)255; };
    CurrentLayout c{};
    c.off_ctl = 0;
    c.off_count = 256;
    c.off_fill = c.off_count + t.n_cells * sizeof(unsigned);
    c.off_offs = a256(c.off_fill + t.n_cells * sizeof(unsigned));
    c.off_bsum = a256(c.off_offs + (t.n_cells + 1) * sizeof(unsigned));
    c.off_base = a256(c.off_bsum + ((t.n_cells + 4095) / 4096) * sizeof(unsigned long long));
    c.off_mask = a256(c.off_base + t.n_cells * 4 * sizeof(unsigned));
    c.off_tables = a256(c.off_mask + (size_t)n_carriers * t.n_chunks * sizeof(unsigned long long));
    c.off_records = a256(c.off_tables + t.n_cols * t.slots * sizeof(int));
    c.fixed_bytes = c.off_records;
    (void)p;
    return c;
}
// Bytes of the four records of one binned event (precision 0: double).
inline size_t current_event_bytes(const Plan& p) { return 4 * (size_t)(p.precision == 0 ? 64 : 32); }
// d_ws may be null (then one wavefront per carrier, no binning).  phase 1:
// zero the output and bin the events; phase 2 (after phase 1 on the same
// stream): accumulate; phases 4 and 3 (each after phase 1, in either order
// or at once): phase 2 without, and with only, the overflow list.  form: 0 binned from kBinnedMinSteps polyline steps
// on, 1 binned whenever there is a workspace, 2 never binned.  max_blocks >
// 0 caps the grids of the largest binning kernels (0: one wavefront per
// carrier and per node column).
hipError_t launch_current(const Plan& p, const void* h, int n_carriers, int n_tracks,
                          const void* pos, const void* charge, const int* track,
                          void* ws, size_t ws_bytes, void* out, hipStream_t s, int phase, int form,
                          int max_blocks = 0);
// Adjoint: lattice-sum derivatives (d/d collocation offset, d/d source width)
// into gd; transposed boundary-fit solves with right-hand sides rhs into lam;
// the event projection to dL/dq(w) (right-hand sides) and the final
// contraction to the parameter gradient.
hipError_t launch_lattice_derivatives(const Plan& p, double* gd, hipStream_t s);
hipError_t launch_field_table_pitch_derivative(const Plan& p, const void* ws, void* out, hipStream_t s);
hipError_t launch_adjoint_solve(const Plan& p, const void* ws, const void* rhs, void* lam, void* rep,
                                hipStream_t s);
hipError_t launch_adjoint_rhs(const Plan& p, const GradLayout& g, const void* ws, int n_carriers,
                              const void* pos, const void* charge, const int* track, const void* grad_i,
                              void* gws, hipStream_t s);
hipError_t launch_adjoint_params(const Plan& p, const GradLayout& g, const void* ws, void* gws, double* out,
                                 hipStream_t s);

// Register-FFT synthesis: N_z = N1 x N2 with both factors at most 32 and
// 2,3,5-smooth.  Pass 1 transforms over N2 (one lane per k1 < N1), pass 2
// over N1.  A schedule is (N_z, N1, samples per staged block); the ones
// wt_h_plan_tune chooses from are listed per size, the default first.
__host__ __device__ constexpr bool synthesis_pow2(int nz) { return nz == 64 || nz == 128 || nz == 256 || nz == 512; }
__host__ __device__ constexpr int synthesis_pow2_n1(int nz) { return nz <= 128 ? 8 : 16; }

struct PipeSchedule {
    int nz, n1, tbc;
};
// Powers of two: 64 = 8 x 8, 128 = 8 x 16, 256 = 16 x 16, 512 = 16 x 32,
// any number of columns up to 4, float or double (a schedule whose buffers
// do not fit in LDS for double is skipped).  Blocks of 8 samples come first:
// they were measured faster on one MI355X (128 x 128 x N_z, 200 samples,
// float H: 0.50 against 0.52 ms at N_z = 64, 0.96 against 1.10 ms at 128,
// 2.12 against 2.52 ms at 256; double: 0.93 against 1.05 ms at 64, 1.99
// against 2.42 ms at 128), more workgroups then sharing a CU.
constexpr PipeSchedule kPow2Schedules[] = {
    {64, 8, 8}, {64, 8, 16}, {128, 8, 8}, {128, 8, 16}, {256, 16, 8}, {256, 16, 16}, {512, 16, 8},
};
constexpr int kNumPow2Schedules = (int)(sizeof(kPow2Schedules) / sizeof(kPow2Schedules[0]));
// The other even 2,3,5-smooth N_z from 72 to 320: float, two columns.
constexpr PipeSchedule kSmoothSchedules[] = {
#include "smooth_schedules.inc"
};
constexpr int kNumSmoothSchedules = (int)(sizeof(kSmoothSchedules) / sizeof(kSmoothSchedules[0]));

// Launch shape of the register-FFT synthesis for N_z = n1 x (N_z / n1),
// blocks of tbc samples and elem bytes per real.
// H is produced in blocks of tbc samples, each staged in LDS as rows of
// 3 x tbc values: sample pair q, component c, real/imaginary part at column
// 6 q + c (+3), plus a gap from pair tbc/4 on; row z at rs z + pad floor(z / N2).
// For the powers of two the gap and the padding keep the transforms' LDS
// accesses free of bank conflicts (two groups of a half-wavefront take sample
// pairs tbc/4 apart); the other sizes use neither.
// Teams: the transform team holds gpw groups of N1 lanes per wavefront (a
// group never straddles two), one group per transform (3 tbc/2 of them); the
// memory team's first ntm_act = (N_z/2) ppt threads own one k_z each and ppt
// sample pairs per pass, rounded up to whole wavefronts.
struct PipeShape {
    int n1, n2, tbc, gap, pad, rs, gpw, ntt, ppt, ntm_act, ntm, threads, buffer;
};
__host__ __device__ constexpr PipeShape pipe_shape_for(int nz, int n1, int tbc) {
    PipeShape s{};
    if (n1 <= 0 || nz % n1 != 0) return s;
    s.n1 = n1;
    s.n2 = nz / s.n1;
    s.tbc = tbc;
    const bool p2 = synthesis_pow2(nz);
    s.gap = p2 ? (tbc == 8 ? 4 : 24) : 0;
    s.pad = p2 ? 3 : 0;
    s.rs = 3 * tbc + s.gap + 1;
    s.gpw = 64 / s.n1;
    const int ng = 3 * (tbc / 2);
    s.ntt = (ng + s.gpw - 1) / s.gpw * 64;
    const int nzh = nz / 2;
    // powers of two: as many pairs per pass as the transform team has
    // threads; other sizes: about 256 memory threads (enough stores in
    // flight for the copy-out)
    int ppt = p2 ? s.ntt / nzh : (256 + nzh / 2) / nzh;
    ppt = ppt > tbc / 2 ? tbc / 2 : ppt;
    s.ppt = ppt < 1 ? 1 : ppt;
    s.ntm_act = nzh * s.ppt;
    s.ntm = (s.ntm_act + 63) / 64 * 64;
    s.threads = s.ntt + s.ntm;
    s.buffer = nz * s.rs + nz / s.n2 * s.pad;
    return s;
}
constexpr size_t kPipeLdsBudget = 160 * 1024;
__host__ __device__ constexpr bool pipe_fits(const PipeShape& s, int elem) {
    return s.n1 > 0 && s.threads <= 1024 && 2 * (size_t)s.buffer * elem <= kPipeLdsBudget;
}
// The k-th schedule of N_z (0: the default) that fits elem bytes per real,
// a shape with n1 = 0 if there is none.
__host__ __device__ constexpr PipeShape pipe_schedule(int nz, int elem, int k) {
    const bool p2 = synthesis_pow2(nz);
    const PipeSchedule* t = p2 ? kPow2Schedules : kSmoothSchedules;
    const int n = p2 ? kNumPow2Schedules : kNumSmoothSchedules;
    for (int i = 0; i < n; ++i) {
        if (t[i].nz != nz) continue;
        const PipeShape s = pipe_shape_for(nz, t[i].n1, t[i].tbc);
        if (!pipe_fits(s, elem)) continue;
        if (k-- == 0) return s;
    }
    return PipeShape{};
}
// Number of schedules of N_z that fit elem bytes per real.
__host__ __device__ constexpr int pipe_schedule_count(int nz, int elem) {
    int n = 0;
    while (pipe_schedule(nz, elem, n).n1 > 0) ++n;
    return n;
}
// LDS bytes of the workgroup (two staging buffers).
inline size_t pipe_lds(const PipeShape& s, size_t re) { return 2 * (size_t)s.buffer * re; }
// Register-FFT synthesis of the smooth sizes (kSmoothSchedules, the plan's
// synth_n1 and synth_tbc): float path, two columns; k_synth_smooth.hip.
hipError_t launch_synthesis_smooth(const Plan& p, char* b, void* h, hipStream_t s);

// Mixed-radix factorisation (radix 4 first, then 2, 3, 5) used by the FFTs.
inline int factorize(int n, int* rad) {
    int k = 0;
    while (n % 4 == 0) { rad[k++] = 4; n /= 4; }
    while (n % 2 == 0) { rad[k++] = 2; n /= 2; }
    while (n % 3 == 0) { rad[k++] = 3; n /= 3; }
    while (n % 5 == 0) { rad[k++] = 5; n /= 5; }
    return n == 1 ? k : -1;
}

}  // namespace wt
