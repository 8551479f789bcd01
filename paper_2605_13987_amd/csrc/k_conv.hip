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
constexpr int kSlots = kConvSlots;     // track accumulators of a workgroup of k_conv_tiles
constexpr int kScanItems = 4096;       // bin counts per workgroup of the scan
constexpr unsigned long long kBinnedMinSteps = 1ull << 24;   // polyline steps from which wt_current bins

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

// An event as one node column of k_conv_tiles uses it: off = byte offset in
// the staged rows of lag 0 - m of its lower z-corner (lane n reads
// off + n * sizeof(Lag4), the upper corner one row further), row = the byte
// offset of that row (lanes before the step read its zero positions);
// info = the accumulator slot of its track (kSlots: none) | 64 if it is the
// last event of its track's run | track << 8; and -q dx times the trilinear
// weights of its two corners in this column.
template <typename T>
struct alignas(16) Staged {
    int off;
    int row;
    int info;
    T g0[3];
    T g1[3];
};
constexpr int kLastOfRun = 64;

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

// One wavefront per (carrier, 64 steps): the bit mask of the steps that are
// events, and one count per event in its bin.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_ev_count(Plan p, ConvTiling tl, int n_carriers, int n_tracks, const T* pos, const int* track,
           unsigned long long* mask, unsigned* count) {
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
    if (lane == 0) mask[wave] = bal;
    if (ev) atomicAdd(count + bin, 1u);
}

// Inclusive scan of one value per thread over the workgroup (LDS scratch of
// one value per wavefront); *total receives the workgroup's sum.
template <typename U>
__device__ inline U block_scan(U v, U* wsum, U* total) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const U u = __shfl_up(v, d, kWave);
        if (lane >= d) v += u;
    }
    if (lane == kWave - 1) wsum[w] = v;
    __syncthreads();
    if (w == 0) {
        U s = lane < nw ? wsum[lane] : (U)0;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const U u = __shfl_up(s, d, kWave);
            if (lane >= d) s += u;
        }
        if (lane < nw) wsum[lane] = s;
        if (lane == nw - 1) *total = s;
    }
    __syncthreads();
    return v + (w > 0 ? wsum[w - 1] : (U)0);
}

// Sum of each workgroup's 4096 bin counts (64-bit).
__global__ void __launch_bounds__(kScanThreads)
k_scan_reduce(const unsigned* count, size_t n, unsigned long long* bsum) {
    __shared__ unsigned long long s[kScanThreads];
    const size_t base = (size_t)blockIdx.x * kScanItems;
    unsigned long long v = 0;
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

// One workgroup: exclusive scan of the block sums in place, the number of
// events, and the overflow flag when they exceed the capacity.
__global__ void __launch_bounds__(kScanThreads)
k_scan_top(unsigned long long* bsum, int nb, unsigned long long* ctl) {
    __shared__ unsigned long long wsum[kScanThreads / kWave];
    __shared__ unsigned long long total;
    unsigned long long carry = 0;
    for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
        const int i = b0 + threadIdx.x;
        const unsigned long long v = i < nb ? bsum[i] : 0ull;
        const unsigned long long inc = block_scan(v, wsum, &total);
        if (i < nb) bsum[i] = carry + inc - v;
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        ctl[0] = carry;
        ctl[1] = carry > ctl[2] ? 1ull : 0ull;
    }
}

// offs[i] = exclusive prefix of count, for i < n; offs[n] = the total
// (32-bit: only used when the events fit the capacity, below 2^32).
__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(const unsigned* count, size_t n, const unsigned long long* bsum, unsigned* offs) {
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
    unsigned run = block_scan(sum, wsum, &total) - sum + (unsigned)bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < per; ++k) {
        if (base + k < n) offs[base + k] = run;
        run += v[k];
    }
    // the thread holding the last bin writes the total after it
    if (base < n && base + per >= n) offs[n] = run;
}

// One wavefront per (carrier, 64 steps) again: every event written into its
// bin (the order inside a bin is not fixed).
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

// Geometry of the staged z-tile of a node column: nodes zb .. zb + ns - 1
// (node N_z read as node 0), time blocks of TB samples (nb of them, the last
// last_len long) of the H layout H[x][y][tb][z][tin][a].
struct TileGeom {
    int zb, ns, nb, TB, last_len;
};

// One (node, time block) unit per thread: its TBC x 3 values, prefetched in
// registers as 16-byte words when the block is full and aligned.
template <int TBC, typename TH>
struct HPrefetch {
    static constexpr int kWords = TBC > 0 ? TBC * 3 * (int)sizeof(TH) / 16 : 1;
    uint4 w[kWords];
    bool full;
};

template <int TBC, typename TH>
__device__ inline const TH* unit_src(const Plan& p, const TH* colH, const TileGeom& g, int s, int tb, int& len) {
    int z = g.zb + s;
    if (z >= p.N[2]) z -= p.N[2];
    len = tb == g.nb - 1 ? g.last_len : g.TB;
    return colH + (size_t)tb * g.TB * p.N[2] * 3 + (size_t)z * len * 3;
}

// The loads are unconditional (a unit that is not a full block loads the
// column's first block instead and is marked not full), so that their
// registers are written by the loads alone and nothing waits for them before
// the next tile commits them.
template <int TBC, typename TH>
__device__ inline void prefetch_h(const Plan& p, const TH* colH, const TileGeom& g, HPrefetch<TBC, TH>& pf) {
    if constexpr (TBC > 0) {
        int s = (int)threadIdx.x % g.ns, tb = (int)threadIdx.x / g.ns;
        pf.full = tb < g.nb && (tb < g.nb - 1 || g.last_len == TBC);
        if (!pf.full) s = tb = 0;                      // block 0 is a full block of TBC samples
        int len;
        const uint4* s4 = reinterpret_cast<const uint4*>(unit_src<TBC>(p, colH, g, s, tb, len));
#pragma unroll
        for (int k = 0; k < HPrefetch<TBC, TH>::kWords; ++k) pf.w[k] = s4[k];
    } else {
        pf.full = false;
    }
}

// Write the tile's lag series into the LDS rows (lag t at row position 64 + t):
// the prefetched unit of this thread from registers, every other unit
// (partial last blocks, unaligned layouts, blocks not a compile-time size)
// value by value from global memory.
template <int TBC, typename TH>
__device__ inline void commit_h(const Plan& p, const ConvTiling& tl, const TH* colH, const TileGeom& g,
                                const HPrefetch<TBC, TH>& pf, Lag4<TH>* hs) {
    const int units = g.ns * g.nb;
    for (int u = threadIdx.x; u < units; u += blockDim.x) {
        const int s = u % g.ns, tb = u / g.ns;
        Lag4<TH>* dst = hs + s * tl.sl + 64 + tb * g.TB;
        if constexpr (TBC > 0) {
            if (u == (int)threadIdx.x && pf.full) {
                union {
                    uint4 w[HPrefetch<TBC, TH>::kWords];
                    TH h[TBC * 3];
                } buf;
#pragma unroll
                for (int k = 0; k < HPrefetch<TBC, TH>::kWords; ++k) buf.w[k] = pf.w[k];
#pragma unroll
                for (int i = 0; i < TBC; ++i) {
                    Lag4<TH> l;
                    l.v[0] = buf.h[3 * i];
                    l.v[1] = buf.h[3 * i + 1];
                    l.v[2] = buf.h[3 * i + 2];
                    l.v[3] = (TH)0;
                    dst[i] = l;
                }
                continue;
            }
        }
        int len;
        const TH* src = unit_src<TBC>(p, colH, g, s, tb, len);
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

// Contribution of a staged event for this lane's sample (nb = the lane's
// byte offset n * sizeof(Lag4), slb = the bytes of one row).
template <typename T, typename TH>
__device__ __attribute__((always_inline)) inline T event_value(const Staged<T>& se, const unsigned char* hs, int nb,
                                                               int slb) {
    const int a0 = max(nb + se.off, se.row);
    T x0, y0, z0, x1, y1, z1;
    load_lag(reinterpret_cast<const Lag4<TH>*>(hs + a0), x0, y0, z0);
    load_lag(reinterpret_cast<const Lag4<TH>*>(hs + a0 + slb), x1, y1, z1);
    T v = se.g0[0] * x0;
    v += se.g0[1] * y0;
    v += se.g0[2] * z0;
    v += se.g1[0] * x1;
    v += se.g1[1] * y1;
    v += se.g1[2] * z1;
    return v;
}

// One workgroup per (node column, range of z-tiles); lanes own output
// samples n = 64 w + lane.  Per z-tile with events: the tile's lag series in
// LDS (prefetched during the previous tile); its events (the four
// neighbouring cell columns' bins), 64 at a time, staged by the first
// wavefront with their two z-corner weights in this column and grouped by
// track with ballots (runs of one track, each with an accumulator slot);
// then every wavefront walks every event, four at a time, and adds a run's
// sum to its track's accumulator in LDS when the run ends (the lanes own
// their samples, so no two lanes touch one accumulator).  The accumulators go
// to the output once, when the workgroup ends.
template <int TBC, typename T, typename TH>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4)))
k_conv_tiles(Plan p, ConvTiling tl, const TH* H, const float* decode, const unsigned* offs, const EvRec<T>* ev,
             const unsigned long long* ctl, int n_tracks, T* out) {
    if (ctl[1] != 0ull) return;                        // the direct form takes these events
    extern __shared__ __align__(16) unsigned char smem[];
    Lag4<TH>* hs = reinterpret_cast<Lag4<TH>*>(smem);                             // [zt + 1][sl]
    Staged<T>* st = reinterpret_cast<Staged<T>*>(smem + tl.lds_h);               // [64]
    T* acc = reinterpret_cast<T*>(smem + tl.lds_h + tl.lds_ev);                  // [kSlots][threads]
    unsigned* boffs = reinterpret_cast<unsigned*>(smem + tl.lds_h + tl.lds_ev + tl.lds_acc);   // [4][tpr + 1]
    __shared__ int s_table[kSlots];
    __shared__ int s_nstaged;

    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & (kWave - 1), w = tid / kWave;
    const int n = tid;                                  // this thread's output sample
    const int nt = p.n_time, Nx = p.N[0], Ny = p.N[1], Nz = p.N[2];
    const int ZT = tl.zt, SL = tl.sl, nzt = tl.n_zt;
    const int col = blockIdx.x / tl.n_zr, zr = blockIdx.x - col * tl.n_zr;
    const int x = col / Ny, y = col - x * Ny;
    const int tA = zr * tl.tpr, tB = min(nzt, tA + tl.tpr), nr = tB - tA;
    if (nr <= 0) return;
    const int R = nr + 1;
    // bin offsets of the four cell columns with a corner on node column
    // (x, y) (q = 2 qx + qy: cell x = x - 1 + qx, cell y = y - 1 + qy), tiles tA .. tB
    for (int i = tid; i < 4 * R; i += nthr) {
        const int q = i / R, k = i - q * R;
        const int cx = (q >> 1) ? x : (x == 0 ? Nx - 1 : x - 1);
        const int cy = (q & 1) ? y : (y == 0 ? Ny - 1 : y - 1);
        boffs[i] = offs[((size_t)cx * Ny + cy) * nzt + tA + k];
    }
    for (int s = tid; s < kSlots; s += nthr) s_table[s] = -1;
    __syncthreads();
    auto count_of = [&](int k) -> unsigned {
        return (boffs[k + 1] - boffs[k]) + (boffs[R + k + 1] - boffs[R + k]) + (boffs[2 * R + k + 1] - boffs[2 * R + k]) +
               (boffs[3 * R + k + 1] - boffs[3 * R + k]);
    };
    if (boffs[nr] - boffs[0] + boffs[R + nr] - boffs[R] + boffs[2 * R + nr] - boffs[2 * R] + boffs[3 * R + nr] -
            boffs[3 * R] ==
        0u)
        return;                                          // no event touches this range
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
#pragma unroll
    for (int s = 0; s < kSlots; ++s) acc[s * nthr + n] = (T)0;
    const TH* colH = H + (size_t)col * Nz * nt * 3;
    const int nb = (nt + p.tb - 1) / p.tb;
    constexpr int LB = (int)sizeof(Lag4<TH>);
    const int slb = SL * LB;
    const int nbyte = n * LB;
    auto geom = [&](int k) {
        TileGeom g;
        g.zb = (tA + k) * ZT;
        g.ns = min(ZT, Nz - g.zb) + 1;
        g.nb = nb;
        g.TB = p.tb;
        g.last_len = nt - (nb - 1) * p.tb;
        return g;
    };
    // event i of tile k: which of the four bins (q), and its record
    auto locate = [&](int k, unsigned i, int& q) -> unsigned {
        const unsigned b0 = boffs[k], b1 = boffs[R + k], b2 = boffs[2 * R + k], b3 = boffs[3 * R + k];
        const unsigned pre1 = boffs[k + 1] - b0;
        const unsigned pre2 = pre1 + (boffs[R + k + 1] - b1);
        const unsigned pre3 = pre2 + (boffs[2 * R + k + 1] - b2);
        q = (i >= pre1) + (i >= pre2) + (i >= pre3);
        return q == 0 ? b0 + i : q == 1 ? b1 + (i - pre1) : q == 2 ? b2 + (i - pre2) : b3 + (i - pre3);
    };
    T dec = (T)1;
    if constexpr (!std::is_same<T, TH>::value) dec = (T)decode[0];

    int k = nr - 1;
    while (k >= 0 && count_of(k) == 0u) --k;
    HPrefetch<TBC, TH> pf;
    prefetch_h<TBC>(p, colH, geom(k), pf);
    // the first wavefront holds the next 64 events of the tile in its lanes
    EvRec<T> rnext;
    int qnext = 0;
    if (w == 0 && (unsigned)lane < count_of(k)) rnext = ev[locate(k, (unsigned)lane, qnext)];
    while (k >= 0) {
        int kn = k - 1;
        while (kn >= 0 && count_of(kn) == 0u) --kn;
        const TileGeom g = geom(k);
        const unsigned E = count_of(k);
        __syncthreads();                                 // the previous tile's rows and events are read
        commit_h<TBC>(p, tl, colH, g, pf, hs);
        if (kn >= 0) prefetch_h<TBC>(p, colH, geom(kn), pf);   // lands while this tile is processed
        for (unsigned e0 = 0; e0 < E; e0 += kWave) {
            if (e0 > 0) __syncthreads();                 // the previous chunk's events are read
            if (w == 0) {
                // stage events e0 .. e0 + 63 of this tile, grouped by track
                const unsigned i = e0 + (unsigned)lane;
                const bool have = i < E;
                EvRec<T> r = rnext;
                int q = qnext;
                if (e0 > 0 && have) r = ev[locate(k, i, q)];
                Staged<T> sr;
                if (have) {
                    const T wx = (q >> 1) ? (T)1 - r.f[0] : r.f[0];
                    const T wy = (q & 1) ? (T)1 - r.f[1] : r.f[1];
                    const T w1 = wx * wy * r.f[2], w0 = wx * wy * ((T)1 - r.f[2]);
                    const int zl = (int)(r.zm & 0xffffu) - g.zb;
                    const int m = (int)(r.zm >> 16);
                    sr.row = zl * slb;
                    sr.off = sr.row + (64 - m) * LB;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        sr.g0[a] = r.g[a] * w0;
                        sr.g1[a] = r.g[a] * w1;
                    }
                }
                const int trk = have ? r.track : -1;
                int tab = lane < kSlots ? s_table[lane] : -2;     // the slot table, one entry per lane
                unsigned long long pending = __ballot(have);
                const unsigned long long lt = (1ull << lane) - 1ull;
                int base = 0, pos = 0;
                while (pending) {
                    const int tk = __builtin_amdgcn_readlane(trk, (int)__builtin_ctzll(pending));
                    const unsigned long long same = __ballot(trk == tk) & pending;
                    const unsigned long long hit = __ballot(tab == tk);
                    int slot;
                    if (hit) {
                        slot = (int)__builtin_ctzll(hit);
                    } else {
                        const unsigned long long fr = __ballot(tab == -1);
                        slot = fr ? (int)__builtin_ctzll(fr) : kSlots;
                        if (slot < kSlots && lane == slot) {
                            tab = tk;
                            s_table[slot] = tk;
                        }
                    }
                    const int cnt = __popcll(same);
                    if ((same >> lane) & 1ull) {
                        pos = base + __popcll(same & lt);
                        sr.info = slot | (pos == base + cnt - 1 ? kLastOfRun : 0) | (tk << 8);
                    }
                    base += cnt;
                    pending &= ~same;
                }
                if (have) st[pos] = sr;
                if (lane == 0) s_nstaged = base;
                // the next 64 events (of this tile, else of the next one)
                const unsigned inext = e0 + kWave + (unsigned)lane;
                if (e0 + kWave < E) {
                    if (inext < E) rnext = ev[locate(k, inext, qnext)];
                } else if (kn >= 0 && (unsigned)lane < count_of(kn)) {
                    rnext = ev[locate(kn, (unsigned)lane, qnext)];
                }
            }
            __syncthreads();
            // every wavefront walks every event, four at a time; a track's
            // sum goes to its accumulator after the last event of its run
            const int ne = s_nstaged;
            const unsigned char* hb = reinterpret_cast<const unsigned char*>(hs);
            T cur = (T)0;
            auto close = [&](int info) {
                if (!(info & kLastOfRun)) return;
                const int slot = info & 63;
                if (slot == kSlots) {                    // a track without a slot
                    if (n < nt && cur != (T)0) atomicAdd(out + (size_t)(info >> 8) * nt + n, cur * dec);
                } else {
                    acc[slot * nthr + n] += cur;
                }
                cur = (T)0;
            };
            int e = 0;
            for (; e + 4 <= ne; e += 4) {
                const Staged<T> s0 = st[e], s1 = st[e + 1], s2 = st[e + 2], s3 = st[e + 3];
                const T v0 = event_value<T, TH>(s0, hb, nbyte, slb), v1 = event_value<T, TH>(s1, hb, nbyte, slb);
                const T v2 = event_value<T, TH>(s2, hb, nbyte, slb), v3 = event_value<T, TH>(s3, hb, nbyte, slb);
                cur += v0;
                close(__builtin_amdgcn_readfirstlane(s0.info));
                cur += v1;
                close(__builtin_amdgcn_readfirstlane(s1.info));
                cur += v2;
                close(__builtin_amdgcn_readfirstlane(s2.info));
                cur += v3;
                close(__builtin_amdgcn_readfirstlane(s3.info));
            }
            for (; e < ne; ++e) {
                const Staged<T> s0 = st[e];
                cur += event_value<T, TH>(s0, hb, nbyte, slb);
                close(__builtin_amdgcn_readfirstlane(s0.info));
            }
        }
        k = kn;
    }
    // the per-track sums of this workgroup
    __syncthreads();
    for (int s = 0; s < kSlots; ++s) {
        const int trk = s_table[s];
        const T v = acc[s * nthr + n];
        if (trk >= 0 && trk < n_tracks && n < nt && v != (T)0) atomicAdd(out + (size_t)trk * nt + n, v * dec);
    }
}

// phase 1: the output zeroed and the events binned; phase 2: the
// accumulation (binned, or the unbinned kernel when the events did not fit
// or there is no workspace).  Phase 2 follows phase 1 on the same stream.
template <typename T, typename TH>
hipError_t current(const Plan& p, const void* h, int n_carriers, int n_tracks, const void* pos, const void* charge,
                   const int* track, void* ws, size_t ws_bytes, void* out, hipStream_t s, int phase, int form) {
    const size_t n_out = (size_t)n_tracks * p.n_time;
    hipError_t e = hipSuccess;
    if (phase == 1) {
        const int zgrid = (int)((n_out + kBlock - 1) / kBlock < 4096 ? (n_out + kBlock - 1) / kBlock : 4096);
        hipLaunchKernelGGL(k_fill_zero<T>, dim3(zgrid > 0 ? zgrid : 1), dim3(kBlock), 0, s, static_cast<T*>(out),
                           n_out);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n_carriers == 0) return e;
    const float* decode = reinterpret_cast<const float*>(static_cast<const char*>(h) + p.h_values_bytes);
    ConvTiling tl = conv_tiling(p, sizeof(TH));
    // 16-byte loads of whole time blocks: H and every block of every column aligned
    tl.vec = (reinterpret_cast<uintptr_t>(h) % 16 == 0 && ((size_t)p.N[2] * p.n_time * 3 * sizeof(TH)) % 16 == 0 &&
              ((size_t)p.tb * 3 * sizeof(TH)) % 16 == 0)
                 ? 1
                 : 0;
    const CurrentLayout cl = current_layout(p, tl, n_carriers);
    static_assert(sizeof(EvRec<float>) == 32 && sizeof(EvRec<double>) == 64, "event record size");
    static_assert(sizeof(Staged<float>) == 48 && sizeof(Staged<double>) == 64, "staged event size");
    // per-bin counts are 32-bit: bin only while every step fits them; below
    // kBinnedMinSteps polyline steps the unbinned kernel is faster (its cost
    // is the steps that move, the binned form's also the grid's columns and
    // tiles: at 2e4 carriers x 200 samples, 0.39 against 1.4 ms on one MI355X)
    const unsigned long long steps = (unsigned long long)n_carriers * p.n_time;
    const bool binned = ws != nullptr && ws_bytes >= cl.fixed_bytes + sizeof(EvRec<T>) && steps < 0xfffffff0ull &&
                        form != 2 && (steps >= kBinnedMinSteps || form == 1);
    unsigned long long* ctl = nullptr;
    if (binned) {
        char* b = static_cast<char*>(ws);
        ctl = reinterpret_cast<unsigned long long*>(b + cl.off_ctl);
        unsigned* count = reinterpret_cast<unsigned*>(b + cl.off_count);
        unsigned* offs = reinterpret_cast<unsigned*>(b + cl.off_offs);
        unsigned long long* bsum = reinterpret_cast<unsigned long long*>(b + cl.off_bsum);
        unsigned long long* mask = reinterpret_cast<unsigned long long*>(b + cl.off_mask);
        EvRec<T>* evs = reinterpret_cast<EvRec<T>*>(b + cl.off_events);
        size_t cap = (ws_bytes - cl.off_events) / sizeof(EvRec<T>);
        if (cap > 0xfffffff0ull) cap = 0xfffffff0ull;
      if (phase == 1) {
        // control words and bin counts are one zero-filled run (no memset
        // nodes, so the sequence can be captured); then the capacity
        const size_t n_zero = (cl.off_count + tl.n_bins * sizeof(unsigned)) / sizeof(unsigned);
        hipLaunchKernelGGL(k_fill_zero<unsigned>, dim3((unsigned)std::min<size_t>((n_zero + kBlock - 1) / kBlock, 4096)),
                           dim3(kBlock), 0, s, reinterpret_cast<unsigned*>(b), n_zero);
        hipLaunchKernelGGL(k_set_capacity, dim3(1), dim3(1), 0, s, ctl, (unsigned long long)cap);
        const size_t waves = (size_t)n_carriers * tl.n_chunks;
        const unsigned grid = (unsigned)((waves + kBlock / kWave - 1) / (kBlock / kWave));
        hipLaunchKernelGGL(k_ev_count<T>, dim3(grid), dim3(kBlock), 0, s, p, tl, n_carriers, n_tracks,
                           static_cast<const T*>(pos), track, mask, count);
        const unsigned nb = (unsigned)((tl.n_bins + kScanItems - 1) / kScanItems);
        hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, count, tl.n_bins, bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, bsum, (int)nb, ctl);
        hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, count, tl.n_bins, bsum, offs);
        hipLaunchKernelGGL(k_ev_scatter<T>, dim3(grid), dim3(kBlock), 0, s, p, tl, n_carriers,
                           static_cast<const T*>(pos), static_cast<const T*>(charge), track, mask, offs, count, ctl,
                           evs);
        return hipGetLastError();
      }
        auto tiles = [&](auto kernel) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)tl.lds_bytes);
            if (e != hipSuccess) return;
            hipLaunchKernelGGL(kernel, dim3((unsigned)((size_t)p.N[0] * p.N[1] * tl.n_zr)), dim3(tl.threads),
                               tl.lds_bytes, s, p, tl, static_cast<const TH*>(h), decode, offs, evs, ctl, n_tracks,
                               static_cast<T*>(out));
        };
        // time blocks of 8 or 16 samples, 16-byte aligned: prefetched in
        // registers, unless a unit is more than 6 words; otherwise staged
        // value by value
        if (tl.vec && p.tb == 16 && 16 * 3 * sizeof(TH) <= 96)
            tiles(k_conv_tiles<16, T, TH>);
        else if (tl.vec && p.tb == 8 && 8 * 3 * sizeof(TH) <= 96)
            tiles(k_conv_tiles<8, T, TH>);
        else
            tiles(k_conv_tiles<0, T, TH>);
        if (e != hipSuccess) return e;
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (phase == 1) return hipSuccess;
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
                          hipStream_t s, int phase, int form) {
    if (p.precision == 0)
        return current<double, double>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s, phase,
                                       form);
    if (p.h_format == 1)
        return current<float, _Float16>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s, phase,
                                        form);
    return current<float, float>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s, phase, form);
}

}  // namespace wt
