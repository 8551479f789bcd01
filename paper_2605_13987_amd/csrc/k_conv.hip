// Induced current, Eq. 1 of the paper (introduction):
//   i(t) = -(q / V_w) int_0^t H(x(t'), t - t') . v(t') dt',  V_w = 1 V,
// discretised on the time grid: every polyline step m of a carrier with a
// non-zero displacement dx (an event) contributes, at every later sample
// n >= m, the field at the step midpoint and lag n - m projected on dx; the
// field between nodes is the trilinear interpolation of the nodal H with
// periodic wrap.
//
// Section 3 of the paper computes the whole correlation of one carrier per
// GPU thread and reads H through the texture cache.  Here the events are
// binned by the grid cell they fall in, and H is read node-column by
// node-column, each node's lag series once:
//
//   k_ev_count    one wavefront per (carrier, 64 steps): which steps move
//                 (a bit mask), and the number of events per bin, a bin being
//                 a grid column of cells times a tile of ZT cells along z;
//   k_scan_*      exclusive scan of the bin counts into bin offsets;
//   k_ev_scatter  the events, written into their bins (lower cell corner,
//                 fractions, -q dx, step, track);
//   k_conv_tiles  one workgroup per block of node columns.  For every node
//                 column and z-tile that some event touches, the lag series
//                 of the tile's ZT + 1 nodes are staged in LDS once; the
//                 events of the four neighbouring cell columns are staged
//                 beside them, sorted by track; lanes own output samples
//                 n = 64 w + lane and accumulate, per track, the two z-corners
//                 of every event that lie in this node column.  Per-track sums
//                 stay in registers until the workgroup ends, then go to the
//                 output with one atomic per sample and track.
//
// Without a workspace, or when the events do not fit the caller's
// workspace, k_current runs instead: one wavefront per carrier, lanes over
// output samples, the 8 corner lag series of each moving step read from
// global memory (decided on the device, so nothing synchronises).
#include "common.hpp"

#include <algorithm>
#include <type_traits>

namespace wt {

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kMaxJ = kMaxTime / kWave;
constexpr int kSlots = 48;             // track accumulators per wavefront of k_conv_tiles
constexpr int kScanItems = 4096;       // bin counts per workgroup of the scan
constexpr int kScanThreads = 1024;

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill_zero(T* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (T)0;
}

template <typename T>
__device__ inline int wrap_index(T f, int n) {
    const T r = f - (T)n * floor(f / (T)n);
    const int i = (int)r;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Lower corner cell and fractions of the midpoint of step m of polyline P,
// and its displacement; false if the step does not move or the midpoint is
// not finite.  The same arithmetic in every kernel, so that the binning and
// the convolution agree on every event.
template <typename T>
__device__ inline bool event_cell(const Plan& p, const T* P, int m, int& x0, int& y0, int& z0, T& fx, T& fy, T& fz,
                                  T& dx, T& dy, T& dz) {
    dx = P[3 * m + 3] - P[3 * m + 0];
    dy = P[3 * m + 4] - P[3 * m + 1];
    dz = P[3 * m + 5] - P[3 * m + 2];
    if (dx == (T)0 && dy == (T)0 && dz == (T)0) return false;
    const T ux = (P[3 * m + 0] + P[3 * m + 3]) * (T)0.5 * (T)(p.N[0] / p.L[0]);
    const T uy = (P[3 * m + 1] + P[3 * m + 4]) * (T)0.5 * (T)(p.N[1] / p.L[1]);
    const T uz = (P[3 * m + 2] + P[3 * m + 5]) * (T)0.5 * (T)(p.N[2] / p.L[2]);
    if (!(isfinite(ux) && isfinite(uy) && isfinite(uz))) return false;
    const T flx = floor(ux), fly = floor(uy), flz = floor(uz);
    fx = ux - flx;
    fy = uy - fly;
    fz = uz - flz;
    // periodic wrap of the lower corner, clamped so every index is in range
    x0 = wrap_index(flx, p.N[0]);
    y0 = wrap_index(fly, p.N[1]);
    z0 = wrap_index(flz, p.N[2]);
    return true;
}

// ---------------------------------------------------------------- one wavefront per carrier

template <typename T>
__device__ inline void flush(T* out, int track, int nt, int lane, T* acc) {
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) {
        const int n = lane + kWave * j;
        if (n < nt && acc[j] != (T)0) atomicAdd(out + (size_t)track * nt + n, acc[j]);
        acc[j] = (T)0;
    }
}

// Two dwords with the alignment of one (an 8-byte load from a 4-byte
// aligned address).
struct alignas(4) Dword2 {
    unsigned lo, hi;
};

// Field of one moving step projected on its displacement, at lag tau, for
// the 8 trilinear corners (weights already carry -q / V_w).  The corner
// columns are held as pointers; offsets inside a column (at most N_z n_time 3
// elements) are 32-bit.
template <typename T, typename TH>
struct Step {
    const TH *c00, *c01, *c10, *c11;   // columns of the 4 (x, y) corners
    int z0, z1;
    T w[8];
    T dx, dy, dz;
};

// TBC: the time block of the H layout when it is a compile-time constant
// (a power of two), else 0 and TB at run time.
template <int TBC, typename T, typename TH>
__device__ inline T step_value(const Step<T, TH>& s, int tau, int TB, int Nz, int last_block, int last_len) {
    const int tbs = TBC > 0 ? TBC : TB;
    const int tb = TBC > 0 ? tau / TBC : tau / TB;
    const int tin = tau - tb * tbs;
    const int len = tb == last_block ? last_len : tbs;
    const unsigned toff = (unsigned)(tb * tbs * Nz * 3 + tin * 3);
    const unsigned o0 = toff + (unsigned)(s.z0 * len * 3), o1 = toff + (unsigned)(s.z1 * len * 3);
    auto proj = [&](const TH* h) {
        if constexpr (std::is_same<TH, _Float16>::value) {
            // the three float16 components with one 8-byte load from the 4-byte
            // aligned word below them (the buffer has at least 2 bytes after
            // its last value); the word is reached by pointer arithmetic on h,
            // so the load stays a global one (a pointer rebuilt from an integer
            // would be flat, and flat loads are waited for with the LDS ones)
            const unsigned odd = (unsigned)(reinterpret_cast<uintptr_t>(h) >> 1) & 1u;
            const Dword2 wv = *reinterpret_cast<const Dword2*>(h - odd);
            const unsigned short e0 = (unsigned short)(wv.lo & 0xffffu), e1 = (unsigned short)(wv.lo >> 16);
            const unsigned short e2 = (unsigned short)(wv.hi & 0xffffu), e3 = (unsigned short)(wv.hi >> 16);
            const T hx = (T)__builtin_bit_cast(_Float16, odd ? e1 : e0);
            const T hy = (T)__builtin_bit_cast(_Float16, odd ? e2 : e1);
            const T hz = (T)__builtin_bit_cast(_Float16, odd ? e3 : e2);
            return hx * s.dx + hy * s.dy + hz * s.dz;
        } else {
            return (T)h[0] * s.dx + (T)h[1] * s.dy + (T)h[2] * s.dz;
        }
    };
    T v = (T)0;
    v += s.w[0] * proj(s.c00 + o0);
    v += s.w[1] * proj(s.c00 + o1);
    v += s.w[2] * proj(s.c01 + o0);
    v += s.w[3] * proj(s.c01 + o1);
    v += s.w[4] * proj(s.c10 + o0);
    v += s.w[5] * proj(s.c10 + o1);
    v += s.w[6] * proj(s.c11 + o0);
    v += s.w[7] * proj(s.c11 + o1);
    return v;
}

template <typename T, typename TH>
__device__ inline bool make_step(const Plan& p, const TH* H, const T* P, int m, T q, Step<T, TH>& s) {
    const int Ny = p.N[1], Nz = p.N[2];
    const size_t col_stride = (size_t)Nz * p.n_time * 3;
    int x0, y0, z0;
    T fx, fy, fz;
    if (!event_cell(p, P, m, x0, y0, z0, fx, fy, fz, s.dx, s.dy, s.dz)) return false;
    const int x1 = x0 + 1 == p.N[0] ? 0 : x0 + 1;
    const int y1 = y0 + 1 == Ny ? 0 : y0 + 1;
    s.z0 = z0;
    s.z1 = z0 + 1 == Nz ? 0 : z0 + 1;
    s.c00 = H + ((size_t)x0 * Ny + y0) * col_stride;
    s.c01 = H + ((size_t)x0 * Ny + y1) * col_stride;
    s.c10 = H + ((size_t)x1 * Ny + y0) * col_stride;
    s.c11 = H + ((size_t)x1 * Ny + y1) * col_stride;
    const T gx = (T)1 - fx, gy = (T)1 - fy, gz = (T)1 - fz;
    // -q folded into the weights (V_w = 1 V)
    s.w[0] = -q * gx * gy * gz;
    s.w[1] = -q * gx * gy * fz;
    s.w[2] = -q * gx * fy * gz;
    s.w[3] = -q * gx * fy * fz;
    s.w[4] = -q * fx * gy * gz;
    s.w[5] = -q * fx * gy * fz;
    s.w[6] = -q * fx * fy * gz;
    s.w[7] = -q * fx * fy * fz;
    return true;
}

// One wavefront per carrier.  Lanes first find the carrier's moving steps (64
// at a time, compacted in LDS by ballot), then run over output samples n =
// lane + 64 j while the wavefront walks the moving steps two at a time.  The
// four wavefronts of a workgroup add their partial currents in LDS before one
// atomic flush when they carry the same track.  H is stored as TH: T, or
// float16 holding H * h_scale, whose sums are scaled by decode = 1 / h_scale
// once per output sample.  Workgroups are dealt to the 8 XCDs round robin,
// so carriers are numbered such that the workgroups resident on one XCD hold
// consecutive carriers, whose common reads its L2 then serves.  With a gate
// (the binned form's control words), the kernel runs only when the binned
// form could not take the events.
template <int TBC, typename T, typename TH>
__global__ void __launch_bounds__(kBlock)
k_current(Plan p, const TH* H, const float* decode, int n_carriers, int n_tracks, const T* pos, const T* charge,
          const int* track, T* out, const unsigned long long* gate) {
    if (gate && gate[1] == 0ull) return;
    __shared__ short steps[kBlock / kWave][kMaxTime];
    __shared__ T part[kBlock / kWave][kMaxTime];
    __shared__ int wtrack[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int nt = p.n_time, TB = p.tb, Nz = p.N[2];
    const int last_block = (nt - 1) / TB;
    const int last_len = nt - last_block * TB;
    const int per_xcd = (gridDim.x + 7) / 8;
    const int c = ((blockIdx.x % 8) * per_xcd + blockIdx.x / 8) * (kBlock / kWave) + wv;

    T acc[kMaxJ];
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) acc[j] = (T)0;
    int tr = -1;
    if (c < n_carriers) {
        tr = track[c];
        if (tr < 0 || tr >= n_tracks) tr = -1;
    }
    if (tr >= 0) {
        const T q = charge[c];
        const T* P = pos + (size_t)c * (nt + 1) * 3;
        // moving steps of this carrier, in order
        int nmov = 0;
        for (int m0 = 0; m0 < nt; m0 += kWave) {
            const int m = m0 + lane;
            bool mv = false;
            if (m < nt) {
                const T dx = P[3 * m + 3] - P[3 * m + 0];
                const T dy = P[3 * m + 4] - P[3 * m + 1];
                const T dz = P[3 * m + 5] - P[3 * m + 2];
                mv = !(dx == (T)0 && dy == (T)0 && dz == (T)0);
            }
            const unsigned long long bal = __ballot(mv);
            if (mv) steps[wv][nmov + __popcll(bal & ((1ull << lane) - 1ull))] = (short)m;
            nmov += __popcll(bal);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int e = 0; e < nmov; e += 2) {
            const int ma = steps[wv][e];
            const int mb = e + 1 < nmov ? steps[wv][e + 1] : -1;
            Step<T, TH> sa, sb;
            const bool va = make_step(p, H, P, ma, q, sa);
            const bool vb = mb >= 0 && make_step(p, H, P, mb, q, sb);
#pragma unroll
            for (int j = 0; j < kMaxJ; ++j) {
                const int n = lane + kWave * j;
                if (n >= nt) continue;
                T v = (T)0;
                if (va && n >= ma) v += step_value<TBC>(sa, n - ma, TB, Nz, last_block, last_len);
                if (vb && n >= mb) v += step_value<TBC>(sb, n - mb, TB, Nz, last_block, last_len);
                acc[j] += v;
            }
        }
    }
    if constexpr (!std::is_same<T, TH>::value) {
        const T dec = (T)decode[0];
#pragma unroll
        for (int j = 0; j < kMaxJ; ++j) acc[j] *= dec;
    }
    // workgroup reduction when all four wavefronts carry the same track
    if (lane == 0) wtrack[wv] = tr;
    __syncthreads();
    bool same = true;
    for (int w = 1; w < kBlock / kWave; ++w) same = same && (wtrack[w] == wtrack[0]);
    if (same && wtrack[0] >= 0) {
#pragma unroll
        for (int j = 0; j < kMaxJ; ++j) {
            const int n = lane + kWave * j;
            if (n < nt) part[wv][n] = acc[j];
        }
        __syncthreads();
        for (int n = threadIdx.x; n < nt; n += kBlock) {
            T v = (T)0;
            for (int w = 0; w < kBlock / kWave; ++w) v += part[w][n];
            if (v != (T)0) atomicAdd(out + (size_t)wtrack[0] * nt + n, v);
        }
    } else if (tr >= 0) {
        flush(out, tr, nt, lane, acc);
    }
}

// ---------------------------------------------------------------- binned form

// An event in global memory: its lower corner z index and step
// (zm = z0 | m << 16), track, fractions inside the cell and -q dx.  The
// cell column is the bin's.
template <typename T>
struct alignas(16) EvRec {
    unsigned zm;
    int track;
    T f[3];
    T g[3];
};

// An event as one node column of k_conv_tiles uses it: slot of its lower
// z-corner in the staged tile and step (zm = zl | m << 16), track, and
// -q dx times the trilinear weights of its two corners in this column.
template <typename T>
struct alignas(16) Staged {
    int zm;
    int track;
    T g0[3];
    T g1[3];
};

// One lag of one staged node: the three components and a zero.
template <typename TH>
struct alignas(4 * sizeof(TH)) Lag4 {
    TH v[4];
};

// The three components of a staged lag, read as one word (8 bytes for
// float16, 16 for float).
template <typename T, typename TH>
__device__ inline void load_lag(const Lag4<TH>* a, T& x, T& y, T& z) {
    if constexpr (std::is_same<TH, _Float16>::value) {
        const uint2 u = *reinterpret_cast<const uint2*>(a);
        x = (T)__builtin_bit_cast(_Float16, (unsigned short)(u.x & 0xffffu));
        y = (T)__builtin_bit_cast(_Float16, (unsigned short)(u.x >> 16));
        z = (T)__builtin_bit_cast(_Float16, (unsigned short)(u.y & 0xffffu));
    } else {
        const Lag4<TH> l = *a;
        x = (T)l.v[0];
        y = (T)l.v[1];
        z = (T)l.v[2];
    }
}

// Workspace control words: [0] number of events, [1] 1 when they do not fit
// (the direct form then runs), [2] the event capacity.
__global__ void k_set_capacity(unsigned long long* ctl, unsigned long long cap) { ctl[2] = cap; }

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_ev_count(Plan p, ConvTiling tl, int n_carriers, int n_tracks, const T* pos, const int* track,
           unsigned long long* mask, unsigned* count, unsigned long long* ctl) {
    const int lane = threadIdx.x & (kWave - 1);
    const size_t wave = (size_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const size_t c = wave / tl.n_chunks;
    if (c >= (size_t)n_carriers) return;
    const int nt = p.n_time;
    const int m = (int)(wave - c * tl.n_chunks) * kWave + lane;
    const int tr = track[c];
    bool ev = false;
    unsigned bin = 0;
    if (tr >= 0 && tr < n_tracks && m < nt) {
        const T* P = pos + c * (size_t)(nt + 1) * 3;
        int x0, y0, z0;
        T fx, fy, fz, dx, dy, dz;
        ev = event_cell(p, P, m, x0, y0, z0, fx, fy, fz, dx, dy, dz);
        bin = ((unsigned)x0 * p.N[1] + y0) * tl.n_zt + z0 / tl.zt;
    }
    const unsigned long long bal = __ballot(ev);
    if (lane == 0) {
        mask[wave] = bal;
        if (bal) atomicAdd(ctl, (unsigned long long)__popcll(bal));
    }
    if (ev) atomicAdd(count + bin, 1u);
}

// Inclusive scan of one value per thread over the workgroup (LDS scratch of
// one int per wavefront, plus one).
__device__ inline unsigned block_scan(unsigned v, unsigned* wsum, unsigned* total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const unsigned u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    if (lane == kWave - 1) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        unsigned s = lane < nw ? wsum[lane] : 0u;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const unsigned u = __shfl_up(s, d, kWave);
            if (lane >= d) s += u;
        }
        if (lane < nw) wsum[lane] = s;
        if (lane == nw - 1) *total = s;
    }
    __syncthreads();
    return v + (w > 0 ? wsum[w - 1] : 0u);
}

__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const unsigned* count, size_t n, unsigned* bsum) {
    __shared__ unsigned s[kScanThreads];
    const size_t base = (size_t)blockIdx.x * kScanItems;
    unsigned v = 0;
    for (int k = 0; k < kScanItems / kScanThreads; ++k) {
        const size_t i = base + (size_t)k * kScanThreads + threadIdx.x;
        if (i < n) v += count[i];
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int h = kScanThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0];
}

// One workgroup: exclusive scan of the block sums in place; the overflow
// flag when the events exceed the capacity.
__global__ void __launch_bounds__(kScanThreads) k_scan_top(unsigned* bsum, int nb, unsigned long long* ctl) {
    __shared__ unsigned wsum[kScanThreads / kWave];
    __shared__ unsigned total;
    unsigned carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int i = b0 + threadIdx.x;
        const unsigned v = i < nb ? bsum[i] : 0u;
        const unsigned inc = block_scan(v, wsum, &total);
        if (i < nb) bsum[i] = carry + inc - v;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) ctl[1] = ctl[0] > ctl[2] ? 1ull : 0ull;
}

// offs[i] = exclusive prefix of count, for i < n; offs[n] = the total.
__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const unsigned* count, size_t n, const unsigned* bsum, unsigned* offs) {
    __shared__ unsigned wsum[kScanThreads / kWave];
    __shared__ unsigned total;
    constexpr int per = kScanItems / kScanThreads;
    const size_t base = (size_t)blockIdx.x * kScanItems + (size_t)threadIdx.x * per;
    unsigned v[per];
    unsigned sum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = base + k < n ? count[base + k] : 0u;
        sum += v[k];
    }
    unsigned run = block_scan(sum, wsum, &total) - sum + bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < per; ++k) {
        if (base + k < n) offs[base + k] = run;
        run += v[k];
    }
    // the thread holding the last bin writes the total after it
    if (base < n && base + per >= n) offs[n] = run;
}

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_ev_scatter(Plan p, ConvTiling tl, int n_carriers, const T* pos, const T* charge, const int* track,
             const unsigned long long* mask, const unsigned* offs, unsigned* count, const unsigned long long* ctl,
             EvRec<T>* ev) {
    const int lane = threadIdx.x & (kWave - 1);
    const size_t wave = (size_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const size_t c = wave / tl.n_chunks;
    if (c >= (size_t)n_carriers) return;
    const unsigned long long bits = mask[wave];
    if (bits == 0ull || ctl[1] != 0ull) return;
    if (!((bits >> lane) & 1ull)) return;
    const int nt = p.n_time;
    const int m = (int)(wave - c * tl.n_chunks) * kWave + lane;
    const T* P = pos + c * (size_t)(nt + 1) * 3;
    int x0, y0, z0;
    T fx, fy, fz, dx, dy, dz;
    if (!event_cell(p, P, m, x0, y0, z0, fx, fy, fz, dx, dy, dz)) return;   // cannot happen: the mask says it moves
    const unsigned bin = ((unsigned)x0 * p.N[1] + y0) * tl.n_zt + z0 / tl.zt;
    const unsigned slot = offs[bin] + atomicSub(count + bin, 1u) - 1u;
    const T q = charge[c];
    EvRec<T> r;
    r.zm = (unsigned)z0 | ((unsigned)m << 16);
    r.track = track[c];
    r.f[0] = fx;
    r.f[1] = fy;
    r.f[2] = fz;
    r.g[0] = -q * dx;
    r.g[1] = -q * dy;
    r.g[2] = -q * dz;
    ev[slot] = r;
}

// The per-track accumulators of a lane are registers: every access below
// uses a compile-time index (recursion instead of loops), so that the array
// is split into registers before any pass could merge the accesses into a
// run-time index (which would put it in scratch memory).
// acc[s] += v for a slot s that is the same on every lane: a switch written
// out in the kernel body (a helper function's cases would be merged into one
// access at a run-time index before it is inlined).
#define WT_SLOT_CASE(k) \
    case k: \
        acc[k] += cur; \
        break;
#define WT_SLOT_CASES8(b)                                                                                           \
    WT_SLOT_CASE(b) WT_SLOT_CASE(b + 1) WT_SLOT_CASE(b + 2) WT_SLOT_CASE(b + 3) WT_SLOT_CASE(b + 4)                 \
    WT_SLOT_CASE(b + 5) WT_SLOT_CASE(b + 6) WT_SLOT_CASE(b + 7)

template <int S, typename T>
__device__ __attribute__((always_inline)) inline void zero_slots(T (&acc)[kSlots]) {
    if constexpr (S < kSlots) {
        acc[S] = (T)0;
        zero_slots<S + 1>(acc);
    }
}

// out[track of slot S][n] += acc[S] * dec for every used slot.
template <int S, typename T>
__device__ __attribute__((always_inline)) inline void flush_slots(const T (&acc)[kSlots], const int* table, int n,
                                                                  int nt, int n_tracks, T dec, T* out) {
    if constexpr (S < kSlots) {
        const int trk = table[S];
        if (trk >= 0 && trk < n_tracks && n < nt && acc[S] != (T)0) atomicAdd(out + (size_t)trk * nt + n, acc[S] * dec);
        flush_slots<S + 1>(acc, table, n, nt, n_tracks, dec, out);
    }
}

// Stage the lag series of nodes z0 .. z0 + ns - 1 (node N_z read as node 0)
// of node column col into LDS rows of SL lags (lag t at row position 64 + t).
// The H layout is time-blocked: block tb of a column holds, for every z, the
// block's len samples x 3 components contiguously.  Full blocks of TBC
// samples whose values are 16-byte aligned (vec) move as 16-byte words.
template <int TBC, typename TH>
__device__ inline void stage_tile(const Plan& p, const ConvTiling& tl, const TH* H, size_t col, int z0, int ns,
                                  Lag4<TH>* hs) {
    const int nt = p.n_time, Nz = p.N[2], TB = p.tb;
    const int nb = (nt + TB - 1) / TB, last_len = nt - (nb - 1) * TB;
    const TH* cb = H + col * (size_t)Nz * nt * 3;
    const int units = ns * nb;
    for (int u = threadIdx.x; u < units; u += blockDim.x) {
        const int s = u % ns, tb = u / ns;
        int z = z0 + s;
        if (z >= Nz) z -= Nz;
        const int len = tb == nb - 1 ? last_len : TB;
        const TH* src = cb + (size_t)tb * TB * Nz * 3 + (size_t)z * len * 3;
        Lag4<TH>* dst = hs + s * tl.sl + 64 + tb * TB;
        constexpr int kVecVals = 16 / sizeof(TH);
        if (TBC > 0 && tl.vec && len == TBC && (TBC * 3) % kVecVals == 0) {
            constexpr int nv = TBC * 3 / kVecVals;
            union {
                uint4 w[nv];
                TH h[TBC * 3];
            } buf;
            const uint4* s4 = reinterpret_cast<const uint4*>(src);
#pragma unroll
            for (int k = 0; k < nv; ++k) buf.w[k] = s4[k];
#pragma unroll
            for (int i = 0; i < TBC; ++i) {
                Lag4<TH> l;
                l.v[0] = buf.h[3 * i];
                l.v[1] = buf.h[3 * i + 1];
                l.v[2] = buf.h[3 * i + 2];
                l.v[3] = (TH)0;
                dst[i] = l;
            }
        } else {
            for (int i = 0; i < len; ++i) {
                Lag4<TH> l;
                l.v[0] = src[3 * i];
                l.v[1] = src[3 * i + 1];
                l.v[2] = src[3 * i + 2];
                l.v[3] = (TH)0;
                dst[i] = l;
            }
        }
    }
}

template <int TBC, typename T, typename TH>
__global__ void __launch_bounds__(512)
k_conv_tiles(Plan p, ConvTiling tl, const TH* H, const float* decode, const unsigned* offs, const EvRec<T>* ev,
             const unsigned long long* ctl, int n_tracks, T* out) {
    if (ctl[1] != 0ull) return;                        // the direct form takes these events
    extern __shared__ __align__(16) unsigned char smem[];
    Lag4<TH>* hs = reinterpret_cast<Lag4<TH>*>(smem);                             // [zt + 1][sl]
    Staged<T>* st = reinterpret_cast<Staged<T>*>(smem + tl.lds_h);               // [threads]
    unsigned* boffs = reinterpret_cast<unsigned*>(smem + tl.lds_h + tl.lds_ev);  // [4][n_zt + 1]
    __shared__ int s_table[kSlots];
    __shared__ int s_cnt[kSlots + 1], s_base[kSlots + 1];
    __shared__ int s_nruns, s_run_key[kSlots + 1], s_run_beg[kSlots + 1], s_run_end[kSlots + 1];

    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int n = tid;                                  // this thread's output sample
    const int nt = p.n_time, Nx = p.N[0], Ny = p.N[1], Nz = p.N[2];
    const int ZT = tl.zt, SL = tl.sl, nzt = tl.n_zt;
    for (int s = tid; s < kSlots; s += nthr) s_table[s] = -1;
    // the lags outside [0, nt) of every staged row read as zero: lanes before
    // an event's step and lanes past the last sample touch them
    for (int i = tid; i < (ZT + 1) * SL; i += nthr) {
        const int lag = i % SL;
        if (lag < 64 || lag >= 64 + nt) {
            Lag4<TH> z;
            z.v[0] = z.v[1] = z.v[2] = z.v[3] = (TH)0;
            hs[i] = z;
        }
    }
    T acc[kSlots];
    zero_slots<0>(acc);
    const int bx = blockIdx.x / tl.nby, by = blockIdx.x - bx * tl.nby;
    const int xe = min(Nx, (bx + 1) * tl.bx), ye = min(Ny, (by + 1) * tl.by);
    for (int x = bx * tl.bx; x < xe; ++x) {
        for (int y = by * tl.by; y < ye; ++y) {
            // the four cell columns with a corner on node column (x, y):
            // q = 2 qx + qy, cell x = x - 1 + qx, cell y = y - 1 + qy
            __syncthreads();
            for (int i = tid; i < 4 * (nzt + 1); i += nthr) {
                const int q = i / (nzt + 1), k = i - q * (nzt + 1);
                const int cx = (q >> 1) ? x : (x == 0 ? Nx - 1 : x - 1);
                const int cy = (q & 1) ? y : (y == 0 ? Ny - 1 : y - 1);
                boffs[i] = offs[((size_t)cx * Ny + cy) * nzt + k];
            }
            __syncthreads();
            for (int zt = nzt - 1; zt >= 0; --zt) {
                // events of the four bins: [pre_q, pre_{q+1}) of the staging order
                const unsigned b0 = boffs[zt], b1 = boffs[(nzt + 1) + zt], b2 = boffs[2 * (nzt + 1) + zt],
                               b3 = boffs[3 * (nzt + 1) + zt];
                const unsigned pre1 = boffs[zt + 1] - b0;
                const unsigned pre2 = pre1 + (boffs[(nzt + 1) + zt + 1] - b1);
                const unsigned pre3 = pre2 + (boffs[2 * (nzt + 1) + zt + 1] - b2);
                const int E = (int)(pre3 + (boffs[3 * (nzt + 1) + zt + 1] - b3));
                if (E == 0) continue;
                const int zb = zt * ZT;
                const int ns = min(ZT, Nz - zb) + 1;
                stage_tile<TBC>(p, tl, H, (size_t)x * Ny + y, zb, ns, hs);
                for (int e0 = 0; e0 < E; e0 += nthr) {
                    if (tid <= kSlots) s_cnt[tid] = 0;
                    __syncthreads();
                    // stage event e0 + tid: its two corners in this column
                    const int i = e0 + tid;
                    int key = 0, rank = 0;
                    Staged<T> sr;
                    if (i < E) {
                        const unsigned ui = (unsigned)i;
                        const int q = (ui >= pre1) + (ui >= pre2) + (ui >= pre3);
                        const unsigned src = q == 0 ? b0 + ui : q == 1 ? b1 + (ui - pre1)
                                                              : q == 2 ? b2 + (ui - pre2) : b3 + (ui - pre3);
                        const EvRec<T> r = ev[src];
                        const T wx = (q >> 1) ? (T)1 - r.f[0] : r.f[0];
                        const T wy = (q & 1) ? (T)1 - r.f[1] : r.f[1];
                        const T w1 = wx * wy * r.f[2], w0 = wx * wy * ((T)1 - r.f[2]);
                        const int zl = (int)(r.zm & 0xffffu) - zb;
                        sr.zm = zl | (int)(r.zm & 0xffff0000u);
                        sr.track = r.track;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            sr.g0[a] = r.g[a] * w0;
                            sr.g1[a] = r.g[a] * w1;
                        }
                        // the track's accumulator slot; slots fill from 0 up
                        int slot = -1;
                        for (int s = 0; s < kSlots; ++s) {
                            const int t = s_table[s];
                            if (t == r.track) {
                                slot = s;
                                break;
                            }
                            if (t == -1) break;
                        }
                        if (slot < 0) {
                            for (int s = 0; s < kSlots; ++s) {
                                const int old = atomicCAS(&s_table[s], -1, r.track);
                                if (old == -1 || old == r.track) {
                                    slot = s;
                                    break;
                                }
                            }
                        }
                        key = slot < 0 ? kSlots : slot;
                        rank = atomicAdd(&s_cnt[key], 1);
                    }
                    __syncthreads();
                    // counting sort by slot: bases and the list of runs
                    if (w == 0) {
                        const int c = lane <= kSlots ? s_cnt[lane] : 0;
                        int incl = c;
#pragma unroll
                        for (int d = 1; d < kWave; d <<= 1) {
                            const int u = __shfl_up(incl, d, kWave);
                            if (lane >= d) incl += u;
                        }
                        if (lane <= kSlots) s_base[lane] = incl - c;
                        const unsigned long long live = __ballot(c > 0);
                        if (c > 0) {
                            const int r = __popcll(live & ((1ull << lane) - 1ull));
                            s_run_key[r] = lane;
                            s_run_beg[r] = incl - c;
                            s_run_end[r] = incl;
                        }
                        if (lane == 0) s_nruns = __popcll(live);
                    }
                    __syncthreads();
                    if (i < E) st[s_base[key] + rank] = sr;
                    __syncthreads();
                    // every wavefront walks every run; lanes own samples
                    const int nruns = s_nruns;
                    const int wlast = __builtin_amdgcn_readfirstlane(kWave * w + kWave - 1);
                    for (int r = 0; r < nruns; ++r) {
                        const int key_r = __builtin_amdgcn_readfirstlane(s_run_key[r]);
                        const int beg = __builtin_amdgcn_readfirstlane(s_run_beg[r]);
                        const int end = __builtin_amdgcn_readfirstlane(s_run_end[r]);
                        const bool spill = key_r == kSlots;     // tracks without a slot
                        T cur = (T)0;
                        for (int k = beg; k < end; ++k) {
                            const Staged<T> e = st[k];
                            const int zm = __builtin_amdgcn_readfirstlane(e.zm);
                            const int m = zm >> 16;
                            if (wlast < m) continue;
                            const int zl = zm & 0xffff;
                            const Lag4<TH>* a = hs + zl * SL + 64 + n - m;
                            T x0, y0, z0, x1, y1, z1;
                            load_lag(a, x0, y0, z0);
                            load_lag(a + SL, x1, y1, z1);
                            T v = e.g0[0] * x0;
                            v += e.g0[1] * y0;
                            v += e.g0[2] * z0;
                            v += e.g1[0] * x1;
                            v += e.g1[1] * y1;
                            v += e.g1[2] * z1;
                            if (spill) {
                                const int trk = __builtin_amdgcn_readfirstlane(e.track);
                                T vv = v;
                                if constexpr (!std::is_same<T, TH>::value) vv *= (T)decode[0];
                                if (n < nt && vv != (T)0) atomicAdd(out + (size_t)trk * nt + n, vv);
                            } else {
                                cur += v;
                            }
                        }
                        static_assert(kSlots == 48, "the switch below lists 48 slots");
                        if (!spill) {
                            switch (key_r) {
                                WT_SLOT_CASES8(0)
                                WT_SLOT_CASES8(8)
                                WT_SLOT_CASES8(16)
                                WT_SLOT_CASES8(24)
                                WT_SLOT_CASES8(32)
                                WT_SLOT_CASES8(40)
                                default: break;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
        }
    }
    // the per-track sums of this workgroup
    __syncthreads();
    T dec = (T)1;
    if constexpr (!std::is_same<T, TH>::value) dec = (T)decode[0];
    flush_slots<0>(acc, s_table, n, nt, n_tracks, dec, out);
}

template <typename T, typename TH>
hipError_t current(const Plan& p, const void* h, int n_carriers, int n_tracks, const void* pos, const void* charge,
                   const int* track, void* ws, size_t ws_bytes, void* out, hipStream_t s) {
    const size_t n_out = (size_t)n_tracks * p.n_time;
    hipError_t e;
    const int zgrid = (int)((n_out + kBlock - 1) / kBlock < 4096 ? (n_out + kBlock - 1) / kBlock : 4096);
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(zgrid > 0 ? zgrid : 1), dim3(kBlock), 0, s, static_cast<T*>(out), n_out);
    e = hipGetLastError();
    if (e != hipSuccess || n_carriers == 0) return e;
    const float* decode = reinterpret_cast<const float*>(static_cast<const char*>(h) + p.h_values_bytes);
    ConvTiling tl = conv_tiling(p, sizeof(TH));
    // 16-byte loads of whole time blocks: H and every block of every column aligned
    tl.vec = (reinterpret_cast<uintptr_t>(h) % 16 == 0 && ((size_t)p.N[2] * p.n_time * 3 * sizeof(TH)) % 16 == 0 &&
              ((size_t)p.tb * 3 * sizeof(TH)) % 16 == 0)
                 ? 1
                 : 0;
    const CurrentLayout cl = current_layout(p, tl, n_carriers);
    const bool binned = ws != nullptr && ws_bytes >= cl.fixed_bytes + sizeof(EvRec<T>);
    static_assert(sizeof(EvRec<float>) == 32 && sizeof(EvRec<double>) == 64, "event record size");
    static_assert(sizeof(Staged<float>) == 32 && sizeof(Staged<double>) == 64, "staged event size");
    unsigned long long* ctl = nullptr;
    if (binned) {
        char* b = static_cast<char*>(ws);
        ctl = reinterpret_cast<unsigned long long*>(b + cl.off_ctl);
        unsigned* count = reinterpret_cast<unsigned*>(b + cl.off_count);
        unsigned* offs = reinterpret_cast<unsigned*>(b + cl.off_offs);
        unsigned* bsum = reinterpret_cast<unsigned*>(b + cl.off_bsum);
        unsigned long long* mask = reinterpret_cast<unsigned long long*>(b + cl.off_mask);
        EvRec<T>* evs = reinterpret_cast<EvRec<T>*>(b + cl.off_events);
        size_t cap = (ws_bytes - cl.off_events) / sizeof(EvRec<T>);
        if (cap > 0xfffffff0ull) cap = 0xfffffff0ull;
        // control words and bin counts are one zero-filled run (no memset
        // nodes, so the sequence can be captured); then the capacity
        const size_t n_zero = (cl.off_count + tl.n_bins * sizeof(unsigned)) / sizeof(unsigned);
        hipLaunchKernelGGL(k_fill_zero<unsigned>, dim3((unsigned)std::min<size_t>((n_zero + kBlock - 1) / kBlock, 4096)),
                           dim3(kBlock), 0, s, reinterpret_cast<unsigned*>(b), n_zero);
        hipLaunchKernelGGL(k_set_capacity, dim3(1), dim3(1), 0, s, ctl, (unsigned long long)cap);
        const size_t waves = (size_t)n_carriers * tl.n_chunks;
        const unsigned grid = (unsigned)((waves + kBlock / kWave - 1) / (kBlock / kWave));
        hipLaunchKernelGGL(k_ev_count<T>, dim3(grid), dim3(kBlock), 0, s, p, tl, n_carriers, n_tracks,
                           static_cast<const T*>(pos), track, mask, count, ctl);
        const unsigned nb = (unsigned)((tl.n_bins + kScanItems - 1) / kScanItems);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, count, tl.n_bins, bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, bsum, (int)nb, ctl);
        hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, count, tl.n_bins, bsum, offs);
        hipLaunchKernelGGL(k_ev_scatter<T>, dim3(grid), dim3(kBlock), 0, s, p, tl, n_carriers,
                           static_cast<const T*>(pos), static_cast<const T*>(charge), track, mask, offs, count, ctl,
                           evs);
        auto tiles = [&](auto kernel) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)tl.lds_bytes);
            if (e != hipSuccess) return;
            hipLaunchKernelGGL(kernel, dim3(tl.nbx * tl.nby), dim3(tl.threads), tl.lds_bytes, s, p, tl,
                               static_cast<const TH*>(h), decode, offs, evs, ctl, n_tracks, static_cast<T*>(out));
        };
        if (p.tb == 16)
            tiles(k_conv_tiles<16, T, TH>);
        else if (p.tb == 8)
            tiles(k_conv_tiles<8, T, TH>);
        else
            tiles(k_conv_tiles<0, T, TH>);
        if (e != hipSuccess) return e;
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // the carriers of workgroup b come from a permutation of [0, 8 * per_xcd)
    // workgroups (some past the last carrier, which then do nothing)
    const int blocks = (n_carriers + kBlock / kWave - 1) / (kBlock / kWave);
    const int grid = 8 * ((blocks + 7) / 8);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, p, static_cast<const TH*>(h), decode, n_carriers,
                           n_tracks, static_cast<const T*>(pos), static_cast<const T*>(charge), track,
                           static_cast<T*>(out), static_cast<const unsigned long long*>(ctl));
    };
    if (p.tb == 16)
        go(k_current<16, T, TH>);
    else if (p.tb == 8)
        go(k_current<8, T, TH>);
    else
        go(k_current<0, T, TH>);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_current(const Plan& p, const void* h, int n_carriers, int n_tracks, const void* pos,
                          const void* charge, const int* track, void* ws, size_t ws_bytes, void* out,
                          hipStream_t s) {
    if (p.precision == 0)
        return current<double, double>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s);
    if (p.h_format == 1)
        return current<float, _Float16>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s);
    return current<float, float>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s);
}

}  // namespace wt
