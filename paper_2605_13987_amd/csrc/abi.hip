// C ABI of the library (declared in include/wt.h): argument validation, plan
// and workspace layout, and the order of the kernel launches.
#include "wt.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "common.hpp"

struct wt_context {
    int device;
    hipStream_t stream;
    std::string last_error;
    bool timing;
    hipEvent_t ev[8];
    int n_events;       // events recorded by the last call
    int stage_ids[8];   // stage id of the interval ending at ev[i+1]
    // wt_h_solve: a second stream (with its fork and join events) on which
    // the field table is built while the boundary fit runs
    hipStream_t aux;
    hipEvent_t aux_fork, aux_join;
    // wt_step: a third stream (and its events) on which the current's
    // binning runs beside the synthesis
    hipStream_t bin;
    hipEvent_t bin_fork, bin_join;
    int n_cu;           // compute units of the device
    // wt_current's form (wt_context_set_current_form)
    int current_form;
    // wt_batch_run: lane streams and their events, made on first use
    int n_lanes;
    hipStream_t lane[WT_MAX_LANES];
    hipEvent_t lane_done[WT_MAX_LANES];
    hipEvent_t fork;
    // wt_h_plan_tune's cache: key (device and grid) -> chosen synthesis launch
    struct TuneEntry {
        int tb, threads, n1, tbc;
        double ms;
    };
    std::string tune_path;
    std::string device_key;
    std::map<std::string, TuneEntry> tune_cache;
};

struct wt_h_plan {
    wt::Plan p;
};

// Workspace of wt_h_solve_static: a static device array, one copy on every
// GPU the library runs on, held until the process ends.  In host code the
// name `scratch` only stands for the symbol; its device address on each GPU
// comes from hipGetSymbolAddress (resolved once per device, with that device
// current, when the first context on it is created) and only that address is
// ever handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[WT_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_resolved[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device); nullptr and
// the runtime's error when it cannot be resolved.
void* static_scratch(int device, hipError_t* err) {
    if (device < 0 || device >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_resolved[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_resolved[device] = true;
    }
    *err = g_scratch_err[device];
    return g_scratch_ptr[device];
}

}  // namespace

namespace {

using wt::Plan;

constexpr int kMaxUnknowns = 528;
constexpr int kStageTables = 0, kStageSolve = 1, kStageTime = 2, kStageFieldTable = 3, kStageSynthesis = 4,
              kStageCurrent = 5, kStageAdjointProjection = 6, kStageAdjointSolve = 7, kStageAdjointParams = 8,
              kStageCurrentBinning = 9;
const char* const kStageNames[] = {"green_tables", "collocation_solve", "time_transform",
                                   "field_table",  "synthesis",         "current",
                                   "adjoint_projection", "adjoint_solve", "adjoint_params", "current_binning"};
// The adjoint's transposed solves use the Schur-complement form of the boundary fit.
constexpr int kMaxGradientCharges = 128;

bool pos_finite(double v) { return std::isfinite(v) && v > 0.0; }

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

wt_status hip_fail(wt_context* ctx, hipError_t e, const char* where) {
    if (ctx) {
        ctx->last_error = std::string(where) + ": " + hipGetErrorString(e);
    }
    return WT_E_HIP;
}

#define WT_HIP(ctx, call, where)                          \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

wt_status validate_and_build(const wt_cell* cell, const wt_column* cols, int n_cols, const wt_spectrum* sp,
                             const wt_h_options* opt, Plan& p) {
    std::memset(&p, 0, sizeof(p));
    if (!cell || !cols || !sp || !opt) return WT_E_INVALID_ARG;
    if (n_cols < 1 || n_cols > wt::kMaxCols) return WT_E_INVALID_ARG;
    const double L[3] = {cell->Lx, cell->Ly, cell->Lz};
    const int N[3] = {cell->Nx, cell->Ny, cell->Nz};
    for (int a = 0; a < 3; ++a) {
        if (!pos_finite(L[a])) return WT_E_INVALID_ARG;
        if (N[a] <= 0) return WT_E_INVALID_ARG;
        if (N[a] < 4 || N[a] > 1024 || (N[a] & 1)) return WT_E_UNSUPPORTED_SIZE;
        p.nrad[a] = wt::factorize(N[a], p.rad[a]);
        if (p.nrad[a] < 0) return WT_E_UNSUPPORTED_SIZE;
        p.L[a] = L[a];
        p.N[a] = N[a];
    }
    if (!pos_finite(cell->eps_r)) return WT_E_INVALID_ARG;
    if (!(cell->sigma_bulk == 0.0)) return WT_E_INVALID_ARG;   // conducting bulk not supported
    if (sp->n_freq < 1 || sp->n_freq > 65535 || sp->n_time < 1) return WT_E_INVALID_ARG;
    if (sp->n_time > wt::kMaxTime) return WT_E_UNSUPPORTED_SIZE;
    if (!pos_finite(sp->dt)) return WT_E_INVALID_ARG;
    if (opt->h_format != WT_H_PLAIN && opt->h_format != WT_H_F16_SCALED) return WT_E_INVALID_ARG;
    if (sp->n_freq > 1 ? !pos_finite(sp->df) : !(std::isfinite(sp->df) && sp->df >= 0.0)) return WT_E_INVALID_ARG;
    if (opt->precision != WT_F64 && opt->precision != WT_F32) return WT_E_INVALID_ARG;
    if (opt->ir_max_iter < 0 || opt->ir_max_iter > 16) return WT_E_INVALID_ARG;
    if (!(std::isfinite(opt->ir_tol) && opt->ir_tol >= 0.0)) return WT_E_INVALID_ARG;
    if (opt->fft_schedule < 0) return WT_E_INVALID_ARG;

    p.eps = cell->eps_r * wt::kEps0;
    p.n_cols = n_cols;
    const double h[3] = {L[0] / N[0], L[1] / N[1], L[2] / N[2]};
    int offset = 0;
    double max_node_spacing = 0.0;
    for (int w = 0; w < n_cols; ++w) {
        const wt_column& c = cols[w];
        if (!std::isfinite(c.x) || !std::isfinite(c.y) || !pos_finite(c.radius) || !std::isfinite(c.z_contact) ||
            !std::isfinite(c.z_free) || !std::isfinite(c.v_applied))
            return WT_E_INVALID_ARG;
        if (c.n_colloc < 2 || c.n_resistivity < 1 || c.n_resistivity > 4) return WT_E_INVALID_ARG;
        double cond = 0.0;
        for (int q = 0; q < c.n_resistivity; ++q) {
            if (!pos_finite(c.resistivity[q])) return WT_E_INVALID_ARG;
            cond += 1.0 / c.resistivity[q];
        }
        if (c.x < 0.0 || c.x >= L[0] || c.y < 0.0 || c.y >= L[1]) return WT_E_GEOMETRY;
        if (c.z_contact < 0.0 || c.z_contact > L[2] || c.z_free < 0.0 || c.z_free > L[2] ||
            c.z_contact == c.z_free)
            return WT_E_GEOMETRY;
        const double fx = c.x / h[0], fy = c.y / h[1];
        if (std::fabs(fx - std::nearbyint(fx)) > 1e-6 || std::fabs(fy - std::nearbyint(fy)) > 1e-6)
            return WT_E_GEOMETRY;
        if (c.radius >= 0.5 * std::fmin(L[0], L[1])) return WT_E_GEOMETRY;
        wt::Column& o = p.col[w];
        o.x = c.x;
        o.y = c.y;
        o.radius = c.radius;
        o.z_contact = c.z_contact;
        o.z_free = c.z_free;
        o.sigma = cond / c.n_resistivity;
        o.n_res = c.n_resistivity;
        for (int q = 0; q < 4; ++q) o.resistivity[q] = q < c.n_resistivity ? c.resistivity[q] : 0.0;
        o.v_applied = c.v_applied;
        o.n = c.n_colloc;
        o.ix = ((int)std::nearbyint(fx)) % N[0];
        o.iy = ((int)std::nearbyint(fy)) % N[1];
        o.offset = offset;
        offset += c.n_colloc;
        o.width = wt::kColWidthFraction * c.radius;
        const double kc = std::sqrt(2.0 * wt::kCutoffExponent) / o.width;
        for (int a = 0; a < 3; ++a) {
            const double mm = std::floor(kc * L[a] / (2.0 * wt::kPi)) + 1.0;
            if (mm > 4096.0) return WT_E_UNSUPPORTED_SIZE;
            o.mmax[a] = (int)mm;
        }
        max_node_spacing = std::fmax(max_node_spacing, std::fabs(c.z_free - c.z_contact) / (c.n_colloc - 1));
    }
    // columns must not overlap: in-plane circles and z ranges both intersecting
    for (int a = 0; a < n_cols; ++a)
        for (int b = a + 1; b < n_cols; ++b) {
            double dx = cols[a].x - cols[b].x, dy = cols[a].y - cols[b].y;
            dx -= L[0] * std::nearbyint(dx / L[0]);
            dy -= L[1] * std::nearbyint(dy / L[1]);
            const double lo_a = std::fmin(cols[a].z_contact, cols[a].z_free), hi_a = std::fmax(cols[a].z_contact, cols[a].z_free);
            const double lo_b = std::fmin(cols[b].z_contact, cols[b].z_free), hi_b = std::fmax(cols[b].z_contact, cols[b].z_free);
            if (std::hypot(dx, dy) < cols[a].radius + cols[b].radius && lo_a <= hi_b && lo_b <= hi_a)
                return WT_E_GEOMETRY;
        }
    p.n_q = offset;
    p.n = offset + 1;
    if (p.n > kMaxUnknowns) return WT_E_UNSUPPORTED_SIZE;

    p.n_freq = sp->n_freq;
    p.n_time = sp->n_time;
    p.df = sp->df;
    p.dt = sp->dt;
    const double nyq = 0.5 / sp->dt;
    p.last_weight_one = (sp->n_freq > 1 && std::fabs(sp->df * (sp->n_freq - 1) - nyq) <= 1e-9 * nyq) ? 1 : 0;
    p.precision = opt->precision;
    p.ir_max_iter = opt->ir_max_iter;
    p.ir_tol = opt->ir_tol;
    p.s_bulk[0] = 1.5 * h[0];
    p.s_bulk[1] = 1.5 * h[1];
    p.s_bulk[2] = std::fmax(1.5 * h[2], max_node_spacing);
    p.nkz_tab = 0;
    for (int w = 0; w < n_cols; ++w) p.nkz_tab = p.nkz_tab > p.col[w].mmax[2] + 1 ? p.nkz_tab : p.col[w].mmax[2] + 1;
    p.nzh = N[2] / 2;

    const size_t re = p.precision == WT_F64 ? sizeof(double) : sizeof(float);
    const size_t cx = 2 * re;
    // Time block of the H layout (the synthesis stages a whole block in LDS):
    // the pipelined register-FFT synthesis where it has a schedule that fits
    // (N_z in {64, 128, 256, 512} with at most 4 columns; the other
    // 2,3,5-smooth sizes of kSmoothSchedules with two columns in float): the
    // size's default schedule, or the one wt_h_options.fft_schedule names;
    // otherwise the LDS Stockham synthesis, whose block is halved until its
    // tables fit.
    const size_t lds_budget = 160 * 1024;
    wt::PipeShape shape{};
    const bool register_form = wt::synthesis_pow2(N[2]) ? n_cols <= 4 : (n_cols == 2 && p.precision == WT_F32);
    if (register_form && wt::pipe_schedule_count(N[2], (int)re) > 0) {
        if (opt->fft_schedule >= wt::pipe_schedule_count(N[2], (int)re)) return WT_E_INVALID_ARG;
        shape = wt::pipe_schedule(N[2], (int)re, opt->fft_schedule);
    }
    if (opt->fft_schedule > 0 && shape.n1 == 0) return WT_E_INVALID_ARG;
    int tb;
    p.synth_n1 = 0;
    p.synth_tbc = 0;
    if (wt::pipe_fits(shape, (int)re) && wt::pipe_lds(shape, re) <= lds_budget) {
        p.synth_kernel = 2;
        p.synth_n1 = shape.n1;
        p.synth_tbc = shape.tbc;
        tb = std::min(sp->n_time, shape.tbc);
    } else {
        // the LDS Stockham synthesis: the largest block (<= 32 samples) whose
        // (3 block + 1) / 2 sample-pair transforms all fit beside the staged
        // block in 40 KB of LDS, so that a block takes one spectrum pass and
        // one FFT and four workgroups share a CU (wt_h_plan_tune refines this)
        p.synth_kernel = 0;
        auto lds_need = [&](int t, int pairs) {
            return (size_t)n_cols * p.nzh * 3 * cx + (size_t)N[2] * t * 3 * re + (size_t)2 * pairs * N[2] * cx;
        };
        const size_t occupancy_budget = 40 * 1024;
        tb = std::min(sp->n_time, 32);
        while (tb > 1 && lds_need(tb, (3 * tb + 1) / 2) > occupancy_budget) tb = (tb + 1) / 2;
        if (lds_need(tb, 1) > lds_budget) return WT_E_UNSUPPORTED_SIZE;
    }
    p.tb = tb;
    p.synth_threads = 256;
    p.h_format = opt->h_format;
    // float16 H is written by the pipelined synthesis only, from the float path
    if (p.h_format == WT_H_F16_SCALED && p.precision != WT_F32) return WT_E_INVALID_ARG;
    if (p.h_format == WT_H_F16_SCALED && p.synth_kernel != 2) return WT_E_UNSUPPORTED_SIZE;

    size_t off = 0;
    for (int a = 0; a < 3; ++a) {
        p.off_tw[a] = off;
        off = align256(off + (size_t)N[a] * cx);
    }
    p.off_g = off;
    off = align256(off + (size_t)n_cols * n_cols * p.nkz_tab * sizeof(double));
    p.off_A = off;
    off = align256(off + (size_t)p.n_q * p.n_q * sizeof(double));
    p.off_lu = off;
    off = align256(off + (size_t)p.n_freq * p.n * p.n * 16);
    p.off_piv = off;
    off = align256(off + (size_t)p.n_freq * p.n * sizeof(int));
    p.off_qw = off;
    off = align256(off + (size_t)p.n_freq * p.n * 16);
    p.off_rep = off;
    off = align256(off + (size_t)p.n_freq * sizeof(wt::SolveReport));
    p.off_qt = off;
    off = align256(off + (size_t)p.n_time * p.n_q * sizeof(double));
    p.off_qhat = off;
    off = align256(off + (size_t)p.n_time * n_cols * p.nzh * cx);
    p.off_ehat = off;
    off = align256(off + (size_t)N[0] * N[1] * p.nzh * 3 * cx);
    p.off_hscale = off;
    off = align256(off + 64 + (size_t)p.nzh * (sizeof(unsigned) + sizeof(float)));
    p.ws_bytes = off;
    const size_t n_h = (size_t)N[0] * N[1] * N[2] * p.n_time * 3;
    if (p.h_format == WT_H_F16_SCALED) {
        p.h_values_bytes = align256(n_h * 2);
        p.h_bytes = p.h_values_bytes + 256;
    } else {
        p.h_values_bytes = n_h * re;
        p.h_bytes = p.h_values_bytes;
    }
    return WT_OK;
}

wt::GradLayout grad_layout(const Plan& p, int n_tracks) {
    wt::GradLayout g{};
    const size_t cx = p.precision == WT_F64 ? 16 : 8;
    g.n_tracks = n_tracks;
    size_t off = 0;
    g.off_phi = off;
    off = align256(off + (size_t)n_tracks * p.n_time * p.n_cols * p.nzh * cx);
    g.off_phis = off;
    off = align256(off + (size_t)n_tracks * p.n_time * p.n_cols * p.nzh * cx);
    g.off_gamma = off;
    off = align256(off + (size_t)p.n_time * p.n_cols * p.nzh * 16);
    g.off_gammas = off;
    off = align256(off + (size_t)p.n_time * p.n_cols * p.nzh * 16);
    g.off_eds = off;
    off = align256(off + (size_t)p.N[0] * p.N[1] * p.nzh * 3 * cx);
    g.off_pitch = off;
    off = align256(off + (size_t)p.n_time * 8);
    g.off_gbar = off;
    off = align256(off + (size_t)p.n_time * p.n_q * 8);
    g.off_rhs = off;
    off = align256(off + (size_t)p.n_freq * p.n * 16);
    g.off_lam = off;
    off = align256(off + (size_t)p.n_freq * p.n * 16);
    g.off_rep = off;
    off = align256(off + (size_t)p.n_freq * sizeof(wt::SolveReport));
    g.off_part = off;
    off = align256(off + (size_t)p.n_freq * p.n_cols * 2 * 8);
    g.off_K = off;
    off = align256(off + (size_t)p.n_q * p.n_q * 8);
    g.off_gd = off;
    off = align256(off + (size_t)3 * p.n_cols * p.n_cols * p.nkz_tab * 8);
    g.off_prod = off;
    off = align256(off + (size_t)3 * p.n_q * p.n_q * 8);
    g.bytes = off;
    return g;
}

void fill_layout(const Plan& p, wt_h_layout* l) {
    l->workspace_bytes = p.ws_bytes;
    l->h_bytes = p.h_bytes;
    l->h_time_block = p.tb;
    l->n_q = p.n_q;
    l->off_A = p.off_A;
    l->off_qw = p.off_qw;
    l->off_qt = p.off_qt;
    l->off_qhat = p.off_qhat;
    l->off_ehat = p.off_ehat;
    l->h_format = p.h_format;
    l->h_decode_offset = p.h_format == WT_H_F16_SCALED ? p.h_values_bytes : 0;
}

wt_status bind(wt_context* ctx) {
    WT_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    return WT_OK;
}

wt_status mark(wt_context* ctx, int stage) {
    if (!ctx->timing) return WT_OK;
    if (ctx->n_events >= 8) return WT_OK;
    WT_HIP(ctx, hipEventRecord(ctx->ev[ctx->n_events], ctx->stream), "hipEventRecord");
    if (ctx->n_events > 0) ctx->stage_ids[ctx->n_events - 1] = stage;
    ++ctx->n_events;
    return WT_OK;
}

// The launches of wt_h_solve on stream s; mark_stage(id) is called after
// each stage (and with -1 before the first).  With fork, the field table
// (which needs only the twiddles and writes only its own part of the
// workspace) is built on the context's second stream while the Green's
// tables, the boundary fit and the time transform run on s; s waits for it
// before the synthesis.  The stage mark of the field table then measures
// only what s still waits for.  before_synthesis() is called right before
// the synthesis launch is enqueued.
template <typename Mark, typename Hook>
wt_status enqueue_solve(wt_context* ctx, const Plan& p, void* ws, void* d_h, hipStream_t s, Mark mark_stage,
                        bool fork, Hook before_synthesis) {
    wt_status st;
    if ((st = mark_stage(-1)) != WT_OK) return st;
    WT_HIP(ctx, wt::launch_twiddles(p, ws, s), "twiddles");
    if (fork) {
        WT_HIP(ctx, hipEventRecord(ctx->aux_fork, s), "hipEventRecord");
        WT_HIP(ctx, hipStreamWaitEvent(ctx->aux, ctx->aux_fork, 0), "hipStreamWaitEvent");
        WT_HIP(ctx, wt::launch_field_table(p, ws, ctx->aux), "field_table");
        WT_HIP(ctx, hipEventRecord(ctx->aux_join, ctx->aux), "hipEventRecord");
    }
    WT_HIP(ctx, wt::launch_green_tables(p, ws, s), "green_tables");
    if ((st = mark_stage(kStageTables)) != WT_OK) return st;
    WT_HIP(ctx, wt::launch_collocation_solve(p, ws, s), "collocation_solve");
    if ((st = mark_stage(kStageSolve)) != WT_OK) return st;
    WT_HIP(ctx, wt::launch_time_transform(p, ws, s), "time_transform");
    if ((st = mark_stage(kStageTime)) != WT_OK) return st;
    if (fork)
        WT_HIP(ctx, hipStreamWaitEvent(s, ctx->aux_join, 0), "hipStreamWaitEvent");
    else
        WT_HIP(ctx, wt::launch_field_table(p, ws, s), "field_table");
    if (p.h_format == WT_H_F16_SCALED) WT_HIP(ctx, wt::launch_h_scale(p, ws, d_h, s), "h_scale");
    if ((st = mark_stage(kStageFieldTable)) != WT_OK) return st;
    if ((st = before_synthesis()) != WT_OK) return st;
    WT_HIP(ctx, wt::launch_synthesis(p, ws, d_h, s), "synthesis");
    return mark_stage(kStageSynthesis);
}

// Key of a tuning result: the device (architecture and compute units) and
// everything of the plan the synthesis launch depends on.
wt_status tune_key(wt_context* ctx, const Plan& p, std::string* key) {
    if (ctx->device_key.empty()) {
        hipDeviceProp_t prop;
        WT_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device), "hipGetDeviceProperties");
        std::string arch = prop.gcnArchName;
        for (char& ch : arch)
            if (ch == ' ') ch = '_';
        ctx->device_key = arch + " " + std::to_string(prop.multiProcessorCount);
    }
    std::ostringstream o;
    o << ctx->device_key << ' ' << p.N[0] << ' ' << p.N[1] << ' ' << p.N[2] << ' ' << p.n_time << ' ' << p.precision
      << ' ' << p.h_format << ' ' << p.n_cols;
    *key = o.str();
    return WT_OK;
}

// Tuning cache file: '#' comment lines, then one line per key:
//   <arch> <CUs> <Nx> <Ny> <Nz> <n_time> <precision> <h_format> <n_cols>  <tb> <threads> <n1> <block> <ms>
bool tune_cache_read(const std::string& path, std::map<std::string, wt_context::TuneEntry>* out) {
    std::ifstream in(path);
    if (!in) return true;                                  // no file yet: an empty cache
    std::string line;
    while (std::getline(in, line)) {
        if (line.empty() || line[0] == '#') continue;
        std::istringstream is(line);
        std::string arch;
        long cus, nx, ny, nz, nt, prec, fmt, nc;
        wt_context::TuneEntry e;
        if (!(is >> arch >> cus >> nx >> ny >> nz >> nt >> prec >> fmt >> nc >> e.tb >> e.threads >> e.n1 >> e.tbc >> e.ms))
            return false;
        std::ostringstream k;
        k << arch << ' ' << cus << ' ' << nx << ' ' << ny << ' ' << nz << ' ' << nt << ' ' << prec << ' ' << fmt << ' '
          << nc;
        (*out)[k.str()] = e;
    }
    return true;
}

bool tune_cache_write(const std::string& path, const std::map<std::string, wt_context::TuneEntry>& cache) {
    const std::string tmp = path + ".tmp";
    {
        std::ofstream o(tmp, std::ios::trunc);
        if (!o) return false;
        o << "# wt_h_plan_tune cache: arch CUs Nx Ny Nz n_time precision h_format n_cols  tb threads n1 block ms\n";
        for (const auto& kv : cache) {
            const auto& e = kv.second;
            o << kv.first << "  " << e.tb << ' ' << e.threads << ' ' << e.n1 << ' ' << e.tbc << ' ' << e.ms << '\n';
        }
        if (!o) return false;
    }
    return std::rename(tmp.c_str(), path.c_str()) == 0;
}

bool carriers_ok(const wt_carriers* car) {
    if (car->n_carriers < 0 || car->n_tracks < 1) return false;
    return car->n_carriers == 0 || (car->d_pos && car->d_charge && car->d_track);
}

// The current computed after the H solve by wt_step.
struct CurrentCall {
    const wt_carriers* car;
    void* ws;
    size_t ws_bytes;
    void* out;
};

// Checks of wt_current's arguments (its workspace may be NULL).
wt_status current_args_ok(const wt_h_plan* plan, const wt_carriers* car, const void* d_workspace,
                          size_t workspace_bytes, const void* d_i_out) {
    if (!car || !d_i_out || !carriers_ok(car)) return WT_E_INVALID_ARG;
    if (d_workspace) {
        if (reinterpret_cast<uintptr_t>(d_workspace) & 255) return WT_E_INVALID_ARG;
        size_t need = 0;
        (void)wt_current_workspace(plan, car->n_carriers, 1, &need);
        if (workspace_bytes < need) return WT_E_WORKSPACE;
    }
    return WT_OK;
}

hipError_t launch_current_phase(const wt_context* ctx, const Plan& p, const void* d_h, const CurrentCall& c,
                                hipStream_t s, int phase, int max_blocks = 0) {
    return wt::launch_current(p, d_h, c.car->n_carriers, c.car->n_tracks, c.car->d_pos, c.car->d_charge,
                              c.car->d_track, c.ws, c.ws ? c.ws_bytes : 0, c.out, s, phase, ctx->current_form,
                              max_blocks);
}

// The accumulation on stream s: the overflow list on the context's third
// stream beside the node-column rows (both only add into the output), joined
// back by an event; under stream capture, one launch sequence on s.
wt_status accumulate(wt_context* ctx, const Plan& p, const void* d_h, const CurrentCall& c, hipStream_t s,
                     bool beside) {
    if (!beside) {
        WT_HIP(ctx, launch_current_phase(ctx, p, d_h, c, s, 2), "current");
        return WT_OK;
    }
    WT_HIP(ctx, hipEventRecord(ctx->bin_fork, s), "hipEventRecord");
    WT_HIP(ctx, hipStreamWaitEvent(ctx->bin, ctx->bin_fork, 0), "hipStreamWaitEvent");
    WT_HIP(ctx, launch_current_phase(ctx, p, d_h, c, ctx->bin, 3), "current overflow");
    WT_HIP(ctx, hipEventRecord(ctx->bin_join, ctx->bin), "hipEventRecord");
    WT_HIP(ctx, launch_current_phase(ctx, p, d_h, c, s, 4), "current");
    WT_HIP(ctx, hipStreamWaitEvent(s, ctx->bin_join, 0), "hipStreamWaitEvent");
    return WT_OK;
}

// Workgroups of the binning kernels beside the synthesis: the fewest that
// still let the binning end within the synthesis, so that the synthesis
// workgroups (one per compute unit at N_z = 512) keep finding room.  At
// 256 x 256 x 512 with 1e6 carriers (400 steps each; 6.5 ms of binning
// alone) one workgroup per unit ends within the synthesis and slows it from
// 36.8 to 40.4 ms; half as many outlast it by 1.8 ms; two per unit slow it
// to 43 ms and uncapped grids to 43-45 ms.  So one workgroup per unit for
// every N_x N_y N_z / 32 carriers.
int bin_beside_blocks(const wt_context* ctx, const Plan& p, int n_carriers) {
    const double nodes = (double)p.N[0] * p.N[1] * p.N[2];
    const double per_cu = std::min(64.0, std::max(1.0, std::ceil(32.0 * n_carriers / nodes)));
    return (int)per_cu * ctx->n_cu;
}

// Body of wt_h_solve and wt_h_solve_static, once the workspace is known, and
// of wt_step (cur != nullptr: the current on the H just written).
wt_status solve_on(wt_context* ctx, const Plan& p, void* d_workspace, void* d_h, wt_h_report* report,
                   const CurrentCall* cur = nullptr) {
    wt_status st = bind(ctx);
    if (st != WT_OK) return st;
    ctx->n_events = 0;
    hipStream_t s = ctx->stream;
    // The field table goes on the second stream only when the boundary fit
    // (one workgroup per frequency, each filling a compute unit) runs in a
    // single round.  With more frequencies than compute units the fit keeps
    // every unit busy and the field table only delays its workgroups
    // (256 x 256 x 512, 512 frequencies: fit 1.04 ms alone, 2.46 ms beside
    // the table; the whole solve 0.4 ms slower forked).  Never under stream
    // capture: a replayed graph ran the forked form slower (3.95 ms against
    // 3.57 ms eager at 128 x 128 x 256) than the sequential one (3.74 ms).
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    WT_HIP(ctx, hipStreamIsCapturing(s, &capture), "hipStreamIsCapturing");
    const bool fork = capture == hipStreamCaptureStatusNone && p.n_freq <= ctx->n_cu;
    // wt_step: the current's binning reads only the carriers, so it runs on
    // the third stream beside the synthesis, which leaves issue slots and
    // registers free on every compute unit (one workgroup per unit at
    // N_z = 512), with grids capped by bin_beside_blocks; it starts after the
    // boundary fit, which needs whole units.  Under stream capture
    // everything stays on the caller's stream.
    const bool beside = cur && capture == hipStreamCaptureStatusNone;
    auto before_synthesis = [&]() -> wt_status {
        if (!beside) return WT_OK;
        WT_HIP(ctx, hipEventRecord(ctx->bin_fork, s), "hipEventRecord");
        WT_HIP(ctx, hipStreamWaitEvent(ctx->bin, ctx->bin_fork, 0), "hipStreamWaitEvent");
        WT_HIP(ctx, launch_current_phase(ctx, p, d_h, *cur, ctx->bin, 1,
                                         bin_beside_blocks(ctx, p, cur->car->n_carriers)),
               "current_binning");
        WT_HIP(ctx, hipEventRecord(ctx->bin_join, ctx->bin), "hipEventRecord");
        return WT_OK;
    };
    st = enqueue_solve(ctx, p, d_workspace, d_h, s, [ctx](int stage) { return mark(ctx, stage); }, fork,
                       before_synthesis);
    if (st != WT_OK) return st;
    if (cur) {
        if (beside)
            WT_HIP(ctx, hipStreamWaitEvent(s, ctx->bin_join, 0), "hipStreamWaitEvent");
        else
            WT_HIP(ctx, launch_current_phase(ctx, p, d_h, *cur, s, 1), "current_binning");
        if ((st = mark(ctx, kStageCurrentBinning)) != WT_OK) return st;
        if ((st = accumulate(ctx, p, d_h, *cur, s, beside)) != WT_OK) return st;
        if ((st = mark(ctx, kStageCurrent)) != WT_OK) return st;
    }
    if (!report) return WT_OK;

    std::vector<wt::SolveReport> rep(p.n_freq);
    WT_HIP(ctx, hipMemcpyAsync(rep.data(), static_cast<char*>(d_workspace) + p.off_rep,
                               rep.size() * sizeof(wt::SolveReport), hipMemcpyDeviceToHost, s),
           "report copy");
    float h_scale = 1.0f;
    if (p.h_format == WT_H_F16_SCALED)
        WT_HIP(ctx, hipMemcpyAsync(&h_scale, static_cast<char*>(d_workspace) + p.off_hscale, sizeof(float),
                                   hipMemcpyDeviceToHost, s),
               "scale copy");
    WT_HIP(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
    report->h_scale = h_scale;
    report->backward_error_max = 0.0;
    report->pivot_ratio_max = 0.0;
    report->ir_iters_max = 0;
    report->singular_count = 0;
    for (const auto& r : rep) {
        report->backward_error_max = std::fmax(report->backward_error_max, r.backward_error);
        report->pivot_ratio_max = std::fmax(report->pivot_ratio_max, r.pivot_ratio);
        report->ir_iters_max = report->ir_iters_max > r.iters ? report->ir_iters_max : r.iters;
        report->singular_count += r.singular ? 1 : 0;
    }
    if (report->singular_count > 0) return WT_E_SINGULAR;
    if (!(report->backward_error_max <= p.ir_tol)) return WT_E_NOT_CONVERGED;
    return WT_OK;
}

}  // namespace

extern "C" {

const char* wt_status_string(wt_status s) {
    switch (s) {
        case WT_OK: return "ok";
        case WT_E_INVALID_ARG: return "invalid argument";
        case WT_E_GEOMETRY: return "invalid geometry";
        case WT_E_UNSUPPORTED_SIZE: return "unsupported size";
        case WT_E_WORKSPACE: return "buffer too small";
        case WT_E_SINGULAR: return "singular collocation system";
        case WT_E_NOT_CONVERGED: return "refinement did not converge";
        case WT_E_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

const char* wt_stage_name(int id) {
    return (id >= 0 && id < (int)(sizeof(kStageNames) / sizeof(kStageNames[0]))) ? kStageNames[id] : "";
}

// Message of the last failed wt_context_create of this thread (no context
// exists to hold it).
static thread_local std::string g_create_error;

wt_status wt_context_create(wt_context** out, int hip_device, void* hip_stream) {
    if (!out) return WT_E_INVALID_ARG;
    *out = nullptr;
    g_create_error.clear();
    int count = 0;
    hipError_t err = hipGetDeviceCount(&count);
    if (err != hipSuccess) {
        g_create_error = std::string("hipGetDeviceCount: ") + hipGetErrorString(err);
        return WT_E_HIP;
    }
    if (hip_device < 0 || hip_device >= count) {
        g_create_error = "no HIP device " + std::to_string(hip_device) + " (" + std::to_string(count) + " visible)";
        return WT_E_HIP;
    }
    err = hipSetDevice(hip_device);
    if (err != hipSuccess) {
        g_create_error = std::string("hipSetDevice: ") + hipGetErrorString(err);
        return WT_E_HIP;
    }
    wt_context* ctx = new (std::nothrow) wt_context();
    if (!ctx) return WT_E_INVALID_ARG;
    ctx->device = hip_device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    ctx->timing = false;
    ctx->n_events = 0;
    for (auto& e : ctx->ev) e = nullptr;
    ctx->n_lanes = 0;
    ctx->fork = nullptr;
    ctx->aux = nullptr;
    ctx->aux_fork = ctx->aux_join = nullptr;
    ctx->bin = nullptr;
    ctx->bin_fork = ctx->bin_join = nullptr;
    ctx->current_form = 0;
    ctx->n_cu = 0;
    if ((err = hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device)) != hipSuccess) {
        g_create_error = std::string("hipDeviceGetAttribute: ") + hipGetErrorString(err);
        delete ctx;
        return WT_E_HIP;
    }
    // the static workspace of wt_h_solve_static on this device (its address
    // is resolved here, once per device; a failure is reported by that call)
    hipError_t scratch_err = hipSuccess;
    (void)static_scratch(hip_device, &scratch_err);
    // the second stream of wt_h_solve (default priority, non-blocking)
    if ((err = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking)) != hipSuccess ||
        (err = hipEventCreateWithFlags(&ctx->aux_fork, hipEventDisableTiming)) != hipSuccess ||
        (err = hipEventCreateWithFlags(&ctx->aux_join, hipEventDisableTiming)) != hipSuccess ||
        (err = hipStreamCreateWithFlags(&ctx->bin, hipStreamNonBlocking)) != hipSuccess ||
        (err = hipEventCreateWithFlags(&ctx->bin_fork, hipEventDisableTiming)) != hipSuccess ||
        (err = hipEventCreateWithFlags(&ctx->bin_join, hipEventDisableTiming)) != hipSuccess) {
        g_create_error = std::string("stream/event creation: ") + hipGetErrorString(err);
        wt_context_destroy(ctx);
        return WT_E_HIP;
    }
    *out = ctx;
    return WT_OK;
}

wt_status wt_context_destroy(wt_context* ctx) {
    if (!ctx) return WT_E_INVALID_ARG;
    for (auto& e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (int l = 0; l < ctx->n_lanes; ++l) {
        (void)hipEventDestroy(ctx->lane_done[l]);
        (void)hipStreamDestroy(ctx->lane[l]);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->aux_fork) (void)hipEventDestroy(ctx->aux_fork);
    if (ctx->aux_join) (void)hipEventDestroy(ctx->aux_join);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->bin_fork) (void)hipEventDestroy(ctx->bin_fork);
    if (ctx->bin_join) (void)hipEventDestroy(ctx->bin_join);
    if (ctx->bin) (void)hipStreamDestroy(ctx->bin);
    delete ctx;
    return WT_OK;
}

const char* wt_context_last_error(const wt_context* ctx) {
    return ctx ? ctx->last_error.c_str() : g_create_error.c_str();
}

wt_status wt_context_enable_timing(wt_context* ctx, int enable) {
    if (!ctx) return WT_E_INVALID_ARG;
    if (enable && !ctx->ev[0]) {
        wt_status st = bind(ctx);
        if (st != WT_OK) return st;
        for (auto& e : ctx->ev) WT_HIP(ctx, hipEventCreate(&e), "hipEventCreate");
    }
    ctx->timing = enable != 0;
    ctx->n_events = 0;
    return WT_OK;
}

wt_status wt_context_stage_times(wt_context* ctx, double* ms, int max_stages, int* stage_ids, int* n_out) {
    if (!ctx || !n_out || (max_stages > 0 && (!ms || !stage_ids))) return WT_E_INVALID_ARG;
    *n_out = 0;
    if (!ctx->timing || ctx->n_events < 2) return WT_OK;
    WT_HIP(ctx, hipEventSynchronize(ctx->ev[ctx->n_events - 1]), "hipEventSynchronize");
    int k = 0;
    for (int i = 0; i + 1 < ctx->n_events && k < max_stages; ++i, ++k) {
        float t = 0.0f;
        WT_HIP(ctx, hipEventElapsedTime(&t, ctx->ev[i], ctx->ev[i + 1]), "hipEventElapsedTime");
        ms[k] = t;
        stage_ids[k] = ctx->stage_ids[i];
    }
    *n_out = k;
    return WT_OK;
}

wt_status wt_h_plan_create(const wt_cell* cell, const wt_column* cols, int n_cols, const wt_spectrum* spectrum,
                           const wt_h_options* options, wt_h_plan** plan, wt_h_layout* layout) {
    if (!plan || !layout) return WT_E_INVALID_ARG;
    *plan = nullptr;
    wt_h_plan* h = new (std::nothrow) wt_h_plan();
    if (!h) return WT_E_INVALID_ARG;
    const wt_status st = validate_and_build(cell, cols, n_cols, spectrum, options, h->p);
    if (st != WT_OK) {
        delete h;
        return st;
    }
    fill_layout(h->p, layout);
    *plan = h;
    return WT_OK;
}

wt_status wt_h_plan_destroy(wt_h_plan* plan) {
    if (!plan) return WT_E_INVALID_ARG;
    delete plan;
    return WT_OK;
}

wt_status wt_h_plan_layout(const wt_h_plan* plan, wt_h_layout* layout) {
    if (!plan || !layout) return WT_E_INVALID_ARG;
    fill_layout(plan->p, layout);
    return WT_OK;
}

wt_status wt_h_solve(wt_context* ctx, const wt_h_plan* plan, void* d_workspace, size_t workspace_bytes, void* d_h,
                     size_t h_bytes, wt_h_report* report) {
    if (!ctx || !plan || !d_workspace || !d_h) return WT_E_INVALID_ARG;
    const Plan& p = plan->p;
    if (workspace_bytes < p.ws_bytes || h_bytes < p.h_bytes) return WT_E_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) || (reinterpret_cast<uintptr_t>(d_h) & 15))
        return WT_E_INVALID_ARG;
    return solve_on(ctx, p, d_workspace, d_h, report);
}

wt_status wt_h_solve_static(wt_context* ctx, const wt_h_plan* plan, void* d_h, size_t h_bytes,
                            wt_h_report* report) {
    if (!ctx || !plan || !d_h) return WT_E_INVALID_ARG;
    const Plan& p = plan->p;
    if (p.ws_bytes > WT_STATIC_WORKSPACE_BYTES) {
        ctx->last_error = "wt_h_solve_static: the plan needs " + std::to_string(p.ws_bytes) +
                          " bytes of workspace; the static workspace holds " +
                          std::to_string((size_t)WT_STATIC_WORKSPACE_BYTES);
        return WT_E_WORKSPACE;
    }
    if (h_bytes < p.h_bytes) return WT_E_WORKSPACE;
    if (reinterpret_cast<uintptr_t>(d_h) & 15) return WT_E_INVALID_ARG;
    wt_status st = bind(ctx);
    if (st != WT_OK) return st;
    hipError_t err = hipSuccess;
    void* ws = static_scratch(ctx->device, &err);
    if (!ws) return hip_fail(ctx, err == hipSuccess ? hipErrorInvalidSymbol : err, "hipGetSymbolAddress(scratch)");
    return solve_on(ctx, p, ws, d_h, report);
}

wt_status wt_context_set_current_form(wt_context* ctx, int form) {
    if (!ctx || form < 0 || form > 2) return WT_E_INVALID_ARG;
    ctx->current_form = form;
    return WT_OK;
}

wt_status wt_current_workspace(const wt_h_plan* plan, int n_carriers, long long max_events, size_t* bytes) {
    if (!plan || !bytes || n_carriers < 0) return WT_E_INVALID_ARG;
    const Plan& p = plan->p;
    const wt::ConvTiling tl = wt::conv_tiling(p);
    const wt::CurrentLayout cl = wt::current_layout(p, tl, n_carriers);
    long long cap = max_events > 0 ? max_events : (long long)n_carriers * p.n_time;
    if (cap < 1) cap = 1;
    *bytes = cl.fixed_bytes + (size_t)cap * wt::current_event_bytes(p);
    return WT_OK;
}

wt_status wt_current(wt_context* ctx, const wt_h_plan* plan, const void* d_h, const wt_carriers* car,
                     void* d_workspace, size_t workspace_bytes, void* d_i_out) {
    if (!ctx || !plan || !d_h) return WT_E_INVALID_ARG;
    wt_status st = current_args_ok(plan, car, d_workspace, workspace_bytes, d_i_out);
    if (st != WT_OK) return st;
    const Plan& p = plan->p;
    if ((st = bind(ctx)) != WT_OK) return st;
    ctx->n_events = 0;
    if ((st = mark(ctx, -1)) != WT_OK) return st;
    const CurrentCall c{car, d_workspace, workspace_bytes, d_i_out};
    WT_HIP(ctx, launch_current_phase(ctx, p, d_h, c, ctx->stream, 1), "current_binning");
    if ((st = mark(ctx, kStageCurrentBinning)) != WT_OK) return st;
    hipStreamCaptureStatus capture = hipStreamCaptureStatusNone;
    WT_HIP(ctx, hipStreamIsCapturing(ctx->stream, &capture), "hipStreamIsCapturing");
    if ((st = accumulate(ctx, p, d_h, c, ctx->stream, capture == hipStreamCaptureStatusNone)) != WT_OK) return st;
    if ((st = mark(ctx, kStageCurrent)) != WT_OK) return st;
    return WT_OK;
}

wt_status wt_step(wt_context* ctx, const wt_h_plan* plan, void* d_workspace, size_t workspace_bytes, void* d_h,
                  size_t h_bytes, const wt_carriers* car, void* d_cur_workspace, size_t cur_workspace_bytes,
                  void* d_i_out, wt_h_report* report) {
    if (!ctx || !plan || !d_workspace || !d_h) return WT_E_INVALID_ARG;
    const Plan& p = plan->p;
    if (workspace_bytes < p.ws_bytes || h_bytes < p.h_bytes) return WT_E_WORKSPACE;
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) || (reinterpret_cast<uintptr_t>(d_h) & 15))
        return WT_E_INVALID_ARG;
    wt_status st = current_args_ok(plan, car, d_cur_workspace, cur_workspace_bytes, d_i_out);
    if (st != WT_OK) return st;
    const CurrentCall c{car, d_cur_workspace, cur_workspace_bytes, d_i_out};
    return solve_on(ctx, p, d_workspace, d_h, report, &c);
}

wt_status wt_context_set_tune_cache(wt_context* ctx, const char* path) {
    if (!ctx) return WT_E_INVALID_ARG;
    ctx->tune_cache.clear();
    ctx->tune_path.clear();
    if (!path || !*path) return WT_OK;
    std::map<std::string, wt_context::TuneEntry> entries;
    if (!tune_cache_read(path, &entries)) {
        ctx->last_error = std::string("tune cache: malformed line in ") + path;
        return WT_E_INVALID_ARG;
    }
    ctx->tune_path = path;
    ctx->tune_cache.swap(entries);
    return WT_OK;
}

int wt_fft_schedule_count(int n_z) { return wt::pipe_schedule_count(n_z, 4); }

wt_status wt_batch_run(wt_context* ctx, int n_items, const wt_batch_item* items, int n_lanes,
                       void* const* d_workspace, size_t workspace_bytes, void* const* d_h, size_t h_bytes,
                       int* item_status) {
    if (!ctx || n_items < 0 || (n_items > 0 && !items) || n_lanes < 1 || n_lanes > WT_MAX_LANES || !d_workspace ||
        !d_h)
        return WT_E_INVALID_ARG;
    for (int l = 0; l < n_lanes; ++l) {
        if (!d_workspace[l] || !d_h[l]) return WT_E_INVALID_ARG;
        if ((reinterpret_cast<uintptr_t>(d_workspace[l]) & 255) || (reinterpret_cast<uintptr_t>(d_h[l]) & 15))
            return WT_E_INVALID_ARG;
    }
    wt_status st = bind(ctx);
    if (st != WT_OK) return st;
    if (!ctx->fork) WT_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming), "hipEventCreate");
    while (ctx->n_lanes < n_lanes) {
        const int l = ctx->n_lanes;
        WT_HIP(ctx, hipStreamCreateWithFlags(&ctx->lane[l], hipStreamNonBlocking), "hipStreamCreate");
        if (hipEventCreateWithFlags(&ctx->lane_done[l], hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(ctx->lane[l]);
            return hip_fail(ctx, hipErrorOutOfMemory, "hipEventCreate");
        }
        ++ctx->n_lanes;
    }
    // per-item checks; then longest first, each to the lane with the least work
    wt_status first_bad = WT_OK;
    std::vector<int> order;
    std::vector<double> cost(n_items, 0.0);
    for (int i = 0; i < n_items; ++i) {
        const wt_batch_item& it = items[i];
        wt_status si = WT_OK;
        if (!it.plan || !it.d_current || !carriers_ok(&it.carriers))
            si = WT_E_INVALID_ARG;
        else if (it.plan->p.ws_bytes > workspace_bytes || it.plan->p.h_bytes > h_bytes)
            si = WT_E_WORKSPACE;
        if (item_status) item_status[i] = si;
        if (si != WT_OK) {
            if (first_bad == WT_OK) first_bad = si;
            continue;
        }
        // seconds at 4 TB/s for H, plus ~1 ms of small launches per item
        cost[i] = (double)it.plan->p.h_bytes / 4e12 + 1e-3;
        order.push_back(i);
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    std::vector<double> load(n_lanes, 0.0);
    std::vector<std::vector<int>> queue(n_lanes);
    for (int i : order) {
        const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[l] += cost[i];
        queue[l].push_back(i);
    }
    WT_HIP(ctx, hipEventRecord(ctx->fork, ctx->stream), "hipEventRecord");
    // A lane that has waited on the fork is joined back into the context's
    // stream before the call returns, also when a later enqueue fails, so
    // that no work is left outside the caller's stream order.
    std::vector<char> forked(n_lanes, 0);
    auto join = [&](int l) -> wt_status {
        WT_HIP(ctx, hipEventRecord(ctx->lane_done[l], ctx->lane[l]), "hipEventRecord");
        WT_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->lane_done[l], 0), "hipStreamWaitEvent");
        forked[l] = 0;
        return WT_OK;
    };
    auto fail = [&](wt_status err) -> wt_status {
        const std::string msg = ctx->last_error;
        for (int l = 0; l < n_lanes; ++l)
            if (forked[l]) (void)join(l);
        ctx->last_error = msg;
        return err;
    };
    for (int l = 0; l < n_lanes; ++l) {
        if (queue[l].empty()) continue;
        hipStream_t s = ctx->lane[l];
        hipError_t e = hipStreamWaitEvent(s, ctx->fork, 0);
        if (e != hipSuccess) return fail(hip_fail(ctx, e, "hipStreamWaitEvent"));
        forked[l] = 1;
        for (int i : queue[l]) {
            const wt_batch_item& it = items[i];
            const Plan& p = it.plan->p;
            st = enqueue_solve(ctx, p, d_workspace[l], d_h[l], s, [](int) { return WT_OK; }, false,
                               []() { return WT_OK; });
            if (st != WT_OK) return fail(st);
            const wt_carriers& c = it.carriers;
            // the lane's workspace is free again once H is written: the
            // current bins its events there (or runs unbinned if it is too small)
            size_t need = 0;
            (void)wt_current_workspace(it.plan, c.n_carriers, 1, &need);
            const bool fits = workspace_bytes >= need;
            for (int phase = 1; phase <= 2 && e == hipSuccess; ++phase)
                e = wt::launch_current(p, d_h[l], c.n_carriers, c.n_tracks, c.d_pos, c.d_charge, c.d_track,
                                       fits ? d_workspace[l] : nullptr, fits ? workspace_bytes : 0, it.d_current, s,
                                       phase, ctx->current_form);
            if (e != hipSuccess) return fail(hip_fail(ctx, e, "current"));
        }
        if ((st = join(l)) != WT_OK) return fail(st);
    }
    return first_bad;
}

wt_status wt_h_plan_tune(wt_context* ctx, wt_h_plan* plan, void* d_workspace, size_t workspace_bytes, void* d_h,
                         size_t h_bytes, wt_tune_report* report) {
    if (!ctx || !plan || !d_workspace || !d_h) return WT_E_INVALID_ARG;
    Plan& p = plan->p;
    if (workspace_bytes < p.ws_bytes || h_bytes < p.h_bytes) return WT_E_WORKSPACE;
    wt_status st = wt_h_solve(ctx, plan, d_workspace, workspace_bytes, d_h, h_bytes, nullptr);
    if (st != WT_OK) return st;
    hipStream_t s = ctx->stream;
    // candidates: the LDS Stockham synthesis's time block (every power of two
    // <= 32 and <= n_time whose staging and one transform pair fit in LDS)
    // and workgroup size; the register-FFT synthesis: the size's schedules
    // (factor N1 and block) that fit
    struct Cand {
        int tb, threads, n1, tbc;
    };
    std::vector<Cand> cands;
    if (p.synth_kernel == 0) {
        const size_t re = p.precision == WT_F64 ? sizeof(double) : sizeof(float);
        const size_t cx = 2 * re;
        for (int t = 32; t >= 1; t /= 2) {
            if (t > p.n_time && t > 1) continue;
            const size_t need = (size_t)p.n_cols * p.nzh * 3 * cx + (size_t)p.N[2] * t * 3 * re + (size_t)2 * p.N[2] * cx;
            if (need > 160 * 1024) continue;
            for (int thr : {256, 512}) cands.push_back({t, thr, 0, 0});
        }
    } else {
        const int elem = p.precision == WT_F64 ? 8 : 4;
        for (int k = 0; k < wt::pipe_schedule_count(p.N[2], elem); ++k) {
            const wt::PipeShape c = wt::pipe_schedule(p.N[2], elem, k);
            cands.push_back({std::min(p.n_time, c.tbc), p.synth_threads, c.n1, c.tbc});
        }
    }
    const Cand start{p.tb, p.synth_threads, p.synth_n1, p.synth_tbc};
    double best_ms = -1.0, start_ms = -1.0;
    Cand best = start;
    auto same = [](const Cand& a, const Cand& b) {
        return a.tb == b.tb && a.threads == b.threads && a.n1 == b.n1 && a.tbc == b.tbc;
    };
    auto apply = [&p](const Cand& c) {
        p.tb = c.tb;
        p.synth_threads = c.threads;
        p.synth_n1 = c.n1;
        p.synth_tbc = c.tbc;
    };
    // a cached result for this device and grid, if it names a candidate
    std::string key;
    bool cached = false;
    if (!ctx->tune_path.empty() && cands.size() > 1) {
        if ((st = tune_key(ctx, p, &key)) != WT_OK) return st;
        const auto it = ctx->tune_cache.find(key);
        if (it != ctx->tune_cache.end()) {
            const Cand c{it->second.tb, it->second.threads, it->second.n1, it->second.tbc};
            for (const Cand& k : cands)
                if (same(k, c)) cached = true;
            if (cached) {
                apply(c);
                best = c;
                best_ms = it->second.ms;
                // H in the cached layout
                WT_HIP(ctx, wt::launch_synthesis(p, d_workspace, d_h, s), "synthesis");
            }
        }
    }
    if (cands.size() > 1 && !cached) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        WT_HIP(ctx, hipEventCreate(&e0), "hipEventCreate");
        hipError_t err = hipEventCreate(&e1);
        for (size_t c = 0; err == hipSuccess && c < cands.size(); ++c) {
            apply(cands[c]);
            err = wt::launch_synthesis(p, d_workspace, d_h, s);                 // warm-up
            if (err == hipSuccess) err = hipEventRecord(e0, s);
            for (int r = 0; r < 2 && err == hipSuccess; ++r) err = wt::launch_synthesis(p, d_workspace, d_h, s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (err != hipSuccess) break;
            const double t = ms / 2.0;
            if (same(cands[c], start)) start_ms = t;
            if (best_ms < 0.0 || t < best_ms) {
                best_ms = t;
                best = cands[c];
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        apply(best);
        if (err != hipSuccess) {
            apply(start);
            return hip_fail(ctx, err, "tune");
        }
        // H in the chosen layout
        WT_HIP(ctx, wt::launch_synthesis(p, d_workspace, d_h, s), "synthesis");
        if (!key.empty()) {
            ctx->tune_cache[key] = wt_context::TuneEntry{best.tb, best.threads, best.n1, best.tbc, best_ms};
            if (!tune_cache_write(ctx->tune_path, ctx->tune_cache)) {
                ctx->last_error = "tune cache: cannot write " + ctx->tune_path;
                return WT_E_INVALID_ARG;
            }
        }
    }
    WT_HIP(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
    if (report) {
        report->n_candidates = cands.size() > 1 ? (int)cands.size() : 1;
        report->h_time_block = p.tb;
        report->threads = p.synth_kernel == 0 ? p.synth_threads
                                              : wt::pipe_shape_for(p.N[2], p.synth_n1, p.synth_tbc).threads;
        report->ms_chosen = best_ms;
        report->ms_default = start_ms;
        report->fft_n1 = p.synth_kernel == 2 ? p.synth_n1 : 0;
        report->from_cache = cached ? 1 : 0;
    }
    return WT_OK;
}

wt_status wt_h_gradient_workspace(const wt_h_plan* plan, int n_tracks, size_t* bytes) {
    if (!plan || !bytes || n_tracks < 1) return WT_E_INVALID_ARG;
    *bytes = 0;
    if (plan->p.n_q > kMaxGradientCharges) return WT_E_UNSUPPORTED_SIZE;
    *bytes = grad_layout(plan->p, n_tracks).bytes;
    return WT_OK;
}

wt_status wt_h_gradient(wt_context* ctx, const wt_h_plan* plan, const void* d_workspace, size_t workspace_bytes,
                        const wt_carriers* car, const void* d_grad_current, void* d_grad_workspace,
                        size_t grad_workspace_bytes, double* d_grad_params, wt_h_report* report) {
    if (!ctx || !plan || !d_workspace || !car || !d_grad_current || !d_grad_workspace || !d_grad_params)
        return WT_E_INVALID_ARG;
    if (car->n_carriers < 0 || car->n_tracks < 1) return WT_E_INVALID_ARG;
    if (car->n_carriers > 0 && (!car->d_pos || !car->d_charge || !car->d_track)) return WT_E_INVALID_ARG;
    const Plan& p = plan->p;
    if (p.n_q > kMaxGradientCharges) return WT_E_UNSUPPORTED_SIZE;
    if ((reinterpret_cast<uintptr_t>(d_workspace) & 255) || (reinterpret_cast<uintptr_t>(d_grad_workspace) & 255))
        return WT_E_INVALID_ARG;
    const wt::GradLayout g = grad_layout(p, car->n_tracks);
    if (workspace_bytes < p.ws_bytes || grad_workspace_bytes < g.bytes) return WT_E_WORKSPACE;
    wt_status st = bind(ctx);
    if (st != WT_OK) return st;
    ctx->n_events = 0;
    hipStream_t s = ctx->stream;
    char* gb = static_cast<char*>(d_grad_workspace);
    if ((st = mark(ctx, -1)) != WT_OK) return st;
    WT_HIP(ctx, wt::launch_lattice_derivatives(p, reinterpret_cast<double*>(gb + g.off_gd), s), "lattice_derivatives");
    WT_HIP(ctx, wt::launch_field_table_pitch_derivative(p, d_workspace, gb + g.off_eds, s), "field_table_derivative");
    WT_HIP(ctx, wt::launch_adjoint_rhs(p, g, d_workspace, car->n_carriers, car->d_pos, car->d_charge, car->d_track,
                                       d_grad_current, d_grad_workspace, s),
           "adjoint_projection");
    if ((st = mark(ctx, kStageAdjointProjection)) != WT_OK) return st;
    WT_HIP(ctx, wt::launch_adjoint_solve(p, d_workspace, gb + g.off_rhs, gb + g.off_lam, gb + g.off_rep, s),
           "adjoint_solve");
    if ((st = mark(ctx, kStageAdjointSolve)) != WT_OK) return st;
    WT_HIP(ctx, wt::launch_adjoint_params(p, g, d_workspace, d_grad_workspace, d_grad_params, s), "adjoint_params");
    if ((st = mark(ctx, kStageAdjointParams)) != WT_OK) return st;
    if (!report) return WT_OK;

    std::vector<wt::SolveReport> rep(p.n_freq);
    WT_HIP(ctx, hipMemcpyAsync(rep.data(), gb + g.off_rep, rep.size() * sizeof(wt::SolveReport),
                               hipMemcpyDeviceToHost, s),
           "report copy");
    WT_HIP(ctx, hipStreamSynchronize(s), "hipStreamSynchronize");
    report->h_scale = 1.0;
    report->backward_error_max = 0.0;
    report->pivot_ratio_max = 0.0;
    report->ir_iters_max = 0;
    report->singular_count = 0;
    for (const auto& r : rep) {
        report->backward_error_max = std::fmax(report->backward_error_max, r.backward_error);
        report->pivot_ratio_max = std::fmax(report->pivot_ratio_max, r.pivot_ratio);
        report->ir_iters_max = report->ir_iters_max > r.iters ? report->ir_iters_max : r.iters;
        report->singular_count += r.singular ? 1 : 0;
    }
    if (report->singular_count > 0) return WT_E_SINGULAR;
    if (!(report->backward_error_max <= p.ir_tol)) return WT_E_NOT_CONVERGED;
    return WT_OK;
}

wt_status wt_electronics(wt_context* ctx, int precision, int n_tracks, int n_time, double dt, const void* d_current,
                         const void* d_response, const void* d_noise, double noise_sigma, double cfd_fraction,
                         void* d_signal, void* d_features) {
    if (!ctx || !d_current || !d_response || !d_signal || !d_features) return WT_E_INVALID_ARG;
    if (precision != WT_F64 && precision != WT_F32) return WT_E_INVALID_ARG;
    if (n_tracks < 1 || n_time < 1 || !pos_finite(dt)) return WT_E_INVALID_ARG;
    if (!(noise_sigma >= 0.0) || !std::isfinite(noise_sigma)) return WT_E_INVALID_ARG;
    if (!(cfd_fraction > 0.0 && cfd_fraction < 1.0)) return WT_E_INVALID_ARG;
    if (n_time > wt::kMaxTime) return WT_E_UNSUPPORTED_SIZE;
    wt_status st = bind(ctx);
    if (st != WT_OK) return st;
    ctx->n_events = 0;
    WT_HIP(ctx, wt::launch_electronics(precision, n_tracks, n_time, dt, d_current, d_response, d_noise, noise_sigma,
                                       cfd_fraction, d_signal, d_features, ctx->stream),
           "electronics");
    return WT_OK;
}

}  // extern "C"
