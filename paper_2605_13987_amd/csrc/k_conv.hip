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
// binned by the grid cell they fall in and H is read node column by node
// column, each needed lag series once:
//
//   k_ev_count     one wavefront per carrier, 64 steps at a time: which steps
//                  move (a bit mask), and the number of events per cell;
//   k_node_count,  records per (node column, z-node): the events of the four
//   k_scan_*       cells around it at that z, scanned into offsets;
//   k_cell_bases   per cell with events, where its records start in each of
//                  the four bins it feeds;
//   k_ev_scatter   every event written as four records, one per corner
//                  column of its cell: step, track and -q dx times the
//                  trilinear weights of its two z-nodes in that column;
//   k_slots        one wavefront per node column: its track table (the
//                  tracks with the most records, the slots of its per-track
//                  sums), and the records of the other tracks copied to an
//                  overflow list;
//   k_conv_rows    one workgroup per node column, one lane per output
//                  sample n.  The column's nodes go through LDS a tile of
//                  z-nodes at a time, as rows of lags (the next tile and the
//                  next records loading meanwhile); for each record every
//                  lane adds the projection at lag n - m of its two z-nodes
//                  to its track's sum, one register per track (records read
//                  into scalar registers, four at a time); the registers go
//                  to the output every thousand or so records;
//   k_conv_overflow the overflow list, one wavefront per record, its two
//                  z-nodes read from global memory.
//
// Without a workspace, or when the records do not fit the caller's
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
constexpr int kScanItems = 4096;       // bin counts per workgroup of the scan
constexpr unsigned long long kBinnedMinSteps = 1ull << 24;   // polyline steps from which wt_current bins

constexpr int kScanThreads = 1024;
constexpr unsigned kFlushRecords = 1024;   // records between flushes of the binned form's per-track sums
constexpr int kOvfRun = 32;                // consecutive overflow entries per wavefront and pass

// Control words of the workspace: [0] records (4 per event), [1] 1 when the
// binned form cannot take the events (the direct form then runs), [2] the
// record capacity, [3] records on the overflow list.
constexpr int kCtlRecords = 0, kCtlFallback = 1, kCtlCapacity = 2, kCtlOverflow = 3;

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
    if (gate && gate[kCtlFallback] == 0ull) return;
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

// A node-column record: one event as seen from one of the four (x, y) corner
// columns of its cell: w0 = its step m | its lower z-node z0 << 16, w1 = its
// track; g0 and g1 are -q dx times the trilinear weights of the event's
// lower and upper z-node in this column.  k_slots rewrites w0 and w1 into
// what the accumulation reads (see there).
// Records are ordered by (node column, lower z-node); inside one such bin by
// the cell they come from, then by arrival.
template <typename T>
struct alignas(sizeof(T) == 8 ? 64 : 32) NodeRec {
    int w0;
    int w1;
    T g[6];
};

// A record whose track is not in its column's table, as the overflow list
// holds it: node column, m | z0 << 16, track, -q dx times the two weights.
template <typename T>
struct alignas(2 * sizeof(NodeRec<T>)) OvfRec {
    int col;
    int zm;
    int track;
    int pad;
    T g[6];
};

__global__ void k_set_capacity(unsigned long long* ctl, unsigned long long cap) { ctl[kCtlCapacity] = cap; }

template <typename T>
__device__ __forceinline__ void ev_count_carrier(const Plan& p, const ConvTiling& tl, size_t c, int n_tracks,
                                                 const T* pos, const int* track, unsigned long long* mask,
                                                 unsigned* count, int lane) {
    const int nt = p.n_time;
    const int tr = track[c];
    const bool valid = tr >= 0 && tr < n_tracks;
    const T* P = pos + c * (size_t)(nt + 1) * 3;
    for (int j = 0; j < tl.n_chunks; ++j) {
        const int m = j * kWave + lane;
        bool ev = false;
        size_t cell = 0;
        if (valid && m < nt) {
            int x0, y0, z0;
            T fx, fy, fz, dx, dy, dz;
            ev = event_cell(p, P, m, x0, y0, z0, fx, fy, fz, dx, dy, dz);
            cell = ((size_t)x0 * p.N[1] + y0) * p.N[2] + z0;
        }
        const unsigned long long bal = __ballot(ev);
        if (lane == 0) mask[c * tl.n_chunks + j] = bal;
        if (ev) atomicAdd(count + cell, 1u);
    }
}

// One wavefront per carrier, 64 steps at a time: the bit mask of the steps
// that are events, and one count per event in its cell.  The wavefronts
// stride over the carriers, so the grid may be smaller than one wavefront
// per carrier (as it is beside the synthesis).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_ev_count(Plan p, ConvTiling tl, int n_carriers, int n_tracks, const T* pos, const int* track,
           unsigned long long* mask, unsigned* count) {
    const int lane = threadIdx.x & (kWave - 1);
    const size_t stride = (size_t)gridDim.x * (kBlock / kWave);
    for (size_t c = (size_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; c < (size_t)n_carriers;
         c += stride)
        ev_count_carrier(p, tl, c, n_tracks, pos, track, mask, count, lane);
}

// Records per (node column, z-node): the events of the four cells that have
// this node column as a corner column, at this z.
__global__ void __launch_bounds__(kBlock)
k_node_count(Plan p, const unsigned* count, unsigned* nodes) {
    const int Nx = p.N[0], Ny = p.N[1], Nz = p.N[2];
    const size_t n = (size_t)Nx * Ny * Nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const size_t col = i / Nz;
        const int z = (int)(i - col * Nz);
        const int X = (int)(col / Ny), Y = (int)(col - (size_t)X * Ny);
        const int Xm = X == 0 ? Nx - 1 : X - 1, Ym = Y == 0 ? Ny - 1 : Y - 1;
        nodes[i] = count[((size_t)X * Ny + Y) * Nz + z] + count[((size_t)X * Ny + Ym) * Nz + z] +
                   count[((size_t)Xm * Ny + Y) * Nz + z] + count[((size_t)Xm * Ny + Ym) * Nz + z];
    }
}

// Per grid cell with events: where its events' records start in each of the
// four bins it feeds (the bins of its corner node columns (x0, y0), (x0,
// y1), (x1, y0), (x1, y1) at its z0): the bin's offset plus the records of
// the cells that come before it in that bin (a bin holds the events of cell
// (X, Y), then (X, Y - 1), (X - 1, Y), (X - 1, Y - 1)).
__global__ void __launch_bounds__(kBlock)
k_cell_bases(Plan p, const unsigned* count, const unsigned* offs, uint4* base) {
    const int Nx = p.N[0], Ny = p.N[1], Nz = p.N[2];
    const size_t n = (size_t)Nx * Ny * Nz;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        if (count[i] == 0) continue;
        const size_t col = i / Nz;
        const int z = (int)(i - col * Nz);
        const int x0 = (int)(col / Ny), y0 = (int)(col - (size_t)x0 * Ny);
        const int x1 = x0 + 1 == Nx ? 0 : x0 + 1, y1 = y0 + 1 == Ny ? 0 : y0 + 1, ym = y0 == 0 ? Ny - 1 : y0 - 1;
        auto cell = [&](int x, int y) { return ((size_t)x * Ny + y) * Nz + z; };
        const unsigned cA = count[cell(x0, y1)], cB = count[cell(x1, y0)], cC = count[cell(x1, ym)],
                       cD = count[cell(x1, y1)];
        base[i] = make_uint4(offs[i], offs[cell(x0, y1)] + cA, offs[cell(x1, y0)] + cB + cC,
                             offs[cell(x1, y1)] + cD + cB + cA);
    }
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

// Sum of each workgroup's 4096 counts (64-bit).
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
// records, and the overflow flag when they exceed the capacity.
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
        ctl[kCtlRecords] = carry;
        ctl[kCtlFallback] = carry > ctl[kCtlCapacity] ? 1ull : 0ull;
    }
}

// In place: the counts become their exclusive prefix (offs[n] = the total;
// 32-bit: only used when the records fit the capacity, below 2^32).  Each
// thread reads its own counts before it writes their offsets.
__global__ void __launch_bounds__(kScanThreads)
k_scan_apply(unsigned* offs, size_t n, const unsigned long long* bsum) {
    __shared__ unsigned wsum[kScanThreads / kWave];
    __shared__ unsigned total;
    constexpr int per = kScanItems / kScanThreads;
    const size_t base = (size_t)blockIdx.x * kScanItems + (size_t)threadIdx.x * per;
    unsigned v[per];
    unsigned sum = 0;
#pragma unroll
    for (int k = 0; k < per; ++k) {
        v[k] = base + k < n ? offs[base + k] : 0u;
        sum += v[k];
    }
    unsigned run = block_scan(sum, wsum, &total) - sum + (unsigned)bsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < per; ++k) {
        if (base + k < n) offs[base + k] = run;
        run += v[k];
    }
    // the thread holding the last count writes the total after it
    if (base < n && base + per >= n) offs[n] = run;
}

// One wavefront per carrier again: every event written as four node-column
// records (w1: the track, until k_slots rewrites it), each at its cell's base
// in that bin (k_cell_bases) plus its arrival index in the cell (fill
// counter).  In the bin of node column (X, Y) and z-node z0 the records of
// cell (X, Y) come first, then those of cells (X, Y - 1), (X - 1, Y) and
// (X - 1, Y - 1).
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_ev_scatter(Plan p, ConvTiling tl, int n_carriers, const T* pos, const T* charge, const int* track,
             const unsigned long long* mask, unsigned* fill, const uint4* base, const unsigned long long* ctl,
             NodeRec<T>* rec) {
    const int lane = threadIdx.x & (kWave - 1);
    if (ctl[kCtlFallback] != 0ull) return;
    const int nt = p.n_time, Ny = p.N[1], Nz = p.N[2];
    const size_t stride = (size_t)gridDim.x * (kBlock / kWave);
    for (size_t c = (size_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave; c < (size_t)n_carriers;
         c += stride) {
        const T* P = pos + c * (size_t)(nt + 1) * 3;
        for (int jc = 0; jc < tl.n_chunks; ++jc) {
            const unsigned long long bits = mask[c * tl.n_chunks + jc];
            if (!((bits >> lane) & 1ull)) continue;
            const int m = jc * kWave + lane;
            int x0, y0, z0;
            T fx, fy, fz, dx, dy, dz;
            // cannot fail: the mask says that this step moves
            if (!event_cell(p, P, m, x0, y0, z0, fx, fy, fz, dx, dy, dz)) continue;
            const size_t cell = ((size_t)x0 * Ny + y0) * Nz + z0;
            const unsigned j = atomicAdd(fill + cell, 1u);
            // where this cell's records start in each of its four bins
            const uint4 bs = base[cell];
            const T q = charge[c];
            const int tr = track[c];
            const T gx = -q * dx, gy = -q * dy, gz = -q * dz;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int ox = k >> 1, oy = k & 1;
                const size_t slot = (size_t)(k == 0 ? bs.x : k == 1 ? bs.y : k == 2 ? bs.z : bs.w) + j;
                const T wxy = (ox ? fx : (T)1 - fx) * (oy ? fy : (T)1 - fy);
                const T w0 = wxy * ((T)1 - fz), w1 = wxy * fz;
                NodeRec<T> r;
                r.w0 = m | (z0 << 16);
                r.w1 = tr;
                r.g[0] = gx * w0;
                r.g[1] = gy * w0;
                r.g[2] = gz * w0;
                r.g[3] = gx * w1;
                r.g[4] = gy * w1;
                r.g[5] = gz * w1;
                rec[slot] = r;
            }
        }
    }
}

// One node column, by one wavefront.  The column's track table: the tl.slots
// tracks with the most records (ties: first appearance; -1 pads it).  Then
// the first two words of every record rewritten for the accumulation, with
// zl = z0 mod tl.zt (its lower z-node inside its tile) and rowb = tl.rl *
// tl.lb (bytes of an LDS row of lags):
//   w0 = zl rowb - m lb    (LDS byte offset of lag -m of its lower node, from
//                           row 0's lag 0)
//   w1 = zl rowb | slot << 24
// A record whose track is past the table takes the spare slot (a sum that
// is never used) and is copied to the overflow list (after the records, in
// the same buffer); when the list would not fit, the direct form takes all
// events (kCtlFallback).
template <typename T>
__device__ __forceinline__ void slots_column(const Plan& p, const ConvTiling& tl, const unsigned* offs,
                                             NodeRec<T>* rec, unsigned long long* ctl, int* tables, size_t col,
                                             int lane) {
    const int S = tl.slots, Nz = p.N[2];
    const unsigned r0 = offs[col * Nz], r1 = offs[col * Nz + Nz];
    // candidates: the column's first 64 distinct tracks (lane i: the i-th)
    // with their record counts
    int cand = -1, cnt = 0, nc = 0;
    for (unsigned b = r0; b < r1; b += kWave) {
        const unsigned r = b + (unsigned)lane;
        const int trk = r < r1 ? rec[r].w1 : -1;             // the track, as k_ev_scatter wrote it
        unsigned long long pending = __ballot(trk >= 0);
        while (pending) {
            const int tk = __builtin_amdgcn_readlane(trk, (int)__builtin_ctzll(pending));
            const unsigned long long same = __ballot(trk == tk);
            pending &= ~same;
            const unsigned long long at = __ballot(cand == tk);
            const int i = at ? (int)__builtin_ctzll(at) : nc;
            if (i < kWave) {
                if (lane == i) {
                    cand = tk;
                    cnt += __popcll(same);
                }
                if (!at) ++nc;
            }
        }
    }
    // the table: the candidates with the most records, most first
    int tab = -1;
    for (int k = 0; k < S; ++k) {
        int best = cnt, who = lane;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const int ob = __shfl_xor(best, d, kWave), ow = __shfl_xor(who, d, kWave);
            if (ob > best || (ob == best && ow < who)) {
                best = ob;
                who = ow;
            }
        }
        if (best <= 0) break;
        const int tk = __builtin_amdgcn_readlane(cand, who);
        if (lane == k) tab = tk;
        if (lane == who) cnt = -1;
    }
    if (lane < S) tables[col * S + lane] = tab;
    const int rowb = tl.rl * tl.lb;
    const unsigned long long total = ctl[kCtlRecords], cap = ctl[kCtlCapacity];
    OvfRec<T>* ovf = reinterpret_cast<OvfRec<T>*>(rec + ((total + 1) & ~1ull));
    const unsigned long long ovf_cap = cap > total + 1 ? (cap - total - 1) / 2 : 0ull;
    for (unsigned b = r0; b < r1; b += kWave) {
        const unsigned r = b + (unsigned)lane;
        const bool have = r < r1;
        const int trk = have ? rec[r].w1 : -1;
        int slot = S;
        unsigned long long pending = __ballot(have);
        while (pending) {
            const int tk = __builtin_amdgcn_readlane(trk, (int)__builtin_ctzll(pending));
            const unsigned long long same = __ballot(trk == tk) & pending;
            const unsigned long long hs = __ballot(tab == tk);
            if ((same >> lane) & 1ull) slot = hs ? (int)__builtin_ctzll(hs) : S;
            pending &= ~same;
        }
        if (!have) continue;
        const int w0 = rec[r].w0, m = w0 & 0xffff, zl = (w0 >> 16) % tl.zt;
        if (slot == S) {
            const unsigned long long i = atomicAdd(ctl + kCtlOverflow, 1ull);
            if (i < ovf_cap) {
                const NodeRec<T> R = rec[r];
                OvfRec<T> o;
                o.col = (int)col;
                o.zm = w0;
                o.track = trk;
                o.pad = 0;
#pragma unroll
                for (int a = 0; a < 6; ++a) o.g[a] = R.g[a];
                ovf[i] = o;
            } else {
                ctl[kCtlFallback] = 1ull;                // no room: the direct form runs
            }
        }
        int2 w;
        w.x = zl * rowb - m * tl.lb;
        w.y = (zl * rowb) | (slot << 24);
        *reinterpret_cast<int2*>(&rec[r].w0) = w;
    }
}

// One wavefront per node column (Strided: the wavefronts stride over the
// columns, for a grid smaller than one wavefront per column).
template <typename T, bool Strided>
__global__ void __launch_bounds__(kBlock)
k_slots(Plan p, ConvTiling tl, const unsigned* offs, NodeRec<T>* rec, unsigned long long* ctl,
        int* tables) {
    const int lane = threadIdx.x & (kWave - 1);
    const size_t first = (size_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (ctl[kCtlFallback] != 0ull) return;
    if constexpr (!Strided) {
        if (first < tl.n_cols) slots_column(p, tl, offs, rec, ctl, tables, first, lane);
    } else {
        for (size_t col = first; col < tl.n_cols; col += (size_t)gridDim.x * (kBlock / kWave))
            slots_column(p, tl, offs, rec, ctl, tables, col, lane);
    }
}

// One node at one lane's lag as loaded: float16 as the 8 bytes from the
// 4-byte aligned word at or below its first value (which holds its three
// values), else the three values.
template <typename TH>
struct LagRaw {
    TH v[3];
};
template <>
struct LagRaw<_Float16> {
    unsigned lo, hi;
};
template <int ZT, typename TH>
struct RawTile {
    LagRaw<TH> n[ZT + 1];
};

// An object in LDS (address space 3), so that accesses stay LDS
// instructions; LDS is read and written through plain and native vector
// types only.
template <typename X>
using Lds = __attribute__((address_space(3))) X;
// An object in the constant address space (4): read-only while the kernel
// runs.
template <typename X>
using Const = __attribute__((address_space(4))) X;
typedef unsigned NU2 __attribute__((ext_vector_type(2)));
typedef unsigned NU4 __attribute__((ext_vector_type(4)));
template <typename X>
using Vec4 = X __attribute__((ext_vector_type(4)));

// One lag of a node in an LDS row: the three components (and one unused).
template <typename TH>
struct alignas(4 * sizeof(TH)) Lag4 {
    TH v[4];
};

// Load this lane's lag of a node (off = byte offset of the lag's first value
// in the column; a float16 buffer has at least 2 bytes after its last value).
template <typename TH>
__device__ inline void load_lag(const unsigned char* colB, unsigned off, LagRaw<TH>& o) {
    if constexpr (std::is_same<TH, _Float16>::value) {
        const NU2 w = *reinterpret_cast<const NU2*>(colB + (off & ~3u));
        o.lo = w.x;
        o.hi = w.y;
    } else {
        const TH* h = reinterpret_cast<const TH*>(colB + off);
        o.v[0] = h[0];
        o.v[1] = h[1];
        o.v[2] = h[2];
    }
}

// A loaded lag as a row entry (sh: for float16, 16 when the lag's values
// start in the high half of the first word, else 0).
template <typename TH>
__device__ __attribute__((always_inline)) inline void store_lag(const LagRaw<TH>& a, unsigned sh, Lds<Lag4<TH>>* dst) {
    if constexpr (std::is_same<TH, _Float16>::value) {
        NU2 w;
        w.x = __builtin_amdgcn_alignbit(a.hi, a.lo, sh);
        w.y = a.hi >> sh;
        *reinterpret_cast<Lds<NU2>*>(dst) = w;
    } else {
        Vec4<TH> l;
        l.x = a.v[0];
        l.y = a.v[1];
        l.z = a.v[2];
        l.w = (TH)0;
        *reinterpret_cast<Lds<Vec4<TH>>*>(dst) = l;
    }
}

// g . H for one row entry, added to v.
template <typename T, typename TH>
__device__ __attribute__((always_inline)) inline T project(const Lds<Lag4<TH>>* src, const T* g, T v) {
    if constexpr (std::is_same<TH, _Float16>::value) {
        const NU2 w = *reinterpret_cast<const Lds<NU2>*>(src);
        v = fma(g[0], (T)__builtin_bit_cast(_Float16, (unsigned short)(w.x & 0xffffu)), v);
        v = fma(g[1], (T)__builtin_bit_cast(_Float16, (unsigned short)(w.x >> 16)), v);
        v = fma(g[2], (T)__builtin_bit_cast(_Float16, (unsigned short)(w.y & 0xffffu)), v);
    } else {
        const Vec4<TH> l = *reinterpret_cast<const Lds<Vec4<TH>>*>(src);
        v = fma(g[0], (T)l.x, v);
        v = fma(g[1], (T)l.y, v);
        v = fma(g[2], (T)l.z, v);
    }
    return v;
}

// A record in scalar registers (read field by field through the constant
// address space; used together, the reads merge into one load).
template <typename T>
struct RecRegs {
    int w0, w1;
    T g[6];
};
template <typename T>
__device__ __attribute__((always_inline)) inline RecRegs<T> record_regs(const Const<NodeRec<T>>* q) {
    RecRegs<T> r;
    r.w0 = q->w0;
    r.w1 = q->w1;
#pragma unroll
    for (int a = 0; a < 6; ++a) r.g[a] = q->g[a];
    return r;
}

// One record's g0 . H(z0) + g1 . H(z0 + 1) at lag n - m (lane_ab: the LDS
// byte address of this lane's lag 0 in row 0; rows_ab: that of row 0's first
// entry; row_b: bytes per row).  Lag n - m of row zl, or the row's first
// (zero) lag when n - m < -64.  The six products are summed first, so that
// the record's term reaches its track's sum with one rounding.
template <typename T, typename TH>
__device__ __attribute__((always_inline)) inline T record_term(unsigned lane_ab, unsigned rows_ab, unsigned row_b,
                                                               const RecRegs<T>& R) {
    const unsigned ab = (unsigned)max((int)lane_ab + R.w0, (int)rows_ab + (R.w1 & 0xffffff));
    const T v = project<T, TH>((const Lds<Lag4<TH>>*)(size_t)ab, R.g, (T)0);
    return project<T, TH>((const Lds<Lag4<TH>>*)(size_t)(ab + row_b), R.g + 3, v);
}

// The per-track sums of one lane: a block of registers indexed with the
// slot (uniform across the wavefront).
template <typename T>
struct SlotSums {
    static constexpr int N = sizeof(T) == 8 ? kConvSlotsF64 : kConvSlotsF32;
    using V = T __attribute__((ext_vector_type(N)));
};

// One workgroup per node column, one lane per output sample n (64
// ceil(n_time / 64) lanes; those past the last sample compute and drop).
// The column's z-nodes go in tiles of ZT: the tile's ZT + 1 nodes are rows of
// lags in LDS (64 zero lags, then lags 0 .. n_time - 1), written by the lanes
// from the lag each loaded (lane tau: lag tau of every node of the tile).
// A record is the same for every lane, so each wavefront reads it from global
// memory into scalar registers; for each record every lane reads lag n - m of
// its two z-nodes and adds g0 . H(z0) + g1 . H(z0 + 1) to the sum of the
// record's track (one register per slot of the column's track table; tracks
// past the table go to the output directly).  Records go four at a time,
// whatever their tracks.  While a tile's records are processed the next
// tile's nodes are in flight, and its records are pulled into the caches.
// The registers go to the output after about every kFlushRecords records,
// one atomic per sample and track.
template <int ZT, typename T, typename TH>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : (sizeof(TH) == 2 ? 6 : 7))))
k_conv_rows(Plan p, ConvTiling tl, const TH* __restrict__ H, const float* __restrict__ decode,
            const unsigned* __restrict__ offs, const NodeRec<T>* __restrict__ rec, const int* __restrict__ tables,
            const unsigned long long* __restrict__ ctl, T* __restrict__ out) {
    if (ctl[kCtlFallback] != 0ull) return;               // the direct form takes these events
    // issue priority above the overflow kernel beside this one (22.12 ->
    // 21.93 ms at 256 x 256 x 512 with float16 H)
    __builtin_amdgcn_s_setprio(3);
    const int Nz = p.N[2], nt = p.n_time;
    const size_t col = blockIdx.x;
    const unsigned* no = offs + col * Nz;
    const unsigned cbeg = no[0];
    if (no[Nz] == cbeg) return;                          // no record in this column
    extern __shared__ __align__(16) unsigned char smem[];
    Lds<unsigned char>* lds = (Lds<unsigned char>*)smem;
    Lds<Lag4<TH>>* rows = reinterpret_cast<Lds<Lag4<TH>>*>(lds);                 // [ZT + 1][RL]
    Lds<unsigned>* zoff = reinterpret_cast<Lds<unsigned>*>(lds + tl.off_zoff);   // [Nz + 1]
    const int tid = threadIdx.x, lane = tid & (kWave - 1), nthr = blockDim.x;
    const int S = tl.slots, RL = tl.rl;
    constexpr unsigned LB = sizeof(Lag4<TH>);
    const unsigned row_b = (unsigned)RL * LB;
    for (int i = tid; i < (ZT + 1) * 64; i += nthr) {
        Lds<NU2>* z = reinterpret_cast<Lds<NU2>*>(rows + (i >> 6) * RL + (i & 63));
#pragma unroll
        for (int w = 0; w < (int)(sizeof(Lag4<TH>) / 8); ++w) z[w] = NU2{0u, 0u};
    }
    for (int i = tid; i <= Nz; i += nthr) zoff[i] = no[i] - cbeg;       // record offsets inside the column
    const int tabv = lane < S ? tables[col * S + lane] : -1;
    // the column's records through the constant address space: read-only
    // for the whole kernel, so uniform reads of them are scalar loads
    const Const<NodeRec<T>>* crec = (const Const<NodeRec<T>>*)(size_t)(rec + cbeg);

    // the lag this lane loads (lanes past the last lag load the last one and
    // do not store it)
    const int tl0 = tid < nt ? tid : nt - 1;
    const int nb = (nt + p.tb - 1) / p.tb;
    const int tb = tl0 / p.tb, tin = tl0 - tb * p.tb;
    const int len = tb == nb - 1 ? nt - (nb - 1) * p.tb : p.tb;
    // byte offsets in the column: this lane's lag of node 0, and from one
    // node to the next
    const unsigned off0 = (unsigned)(tb * p.tb * Nz * 3 + tin * 3) * (unsigned)sizeof(TH);
    const unsigned zs_b = (unsigned)(len * 3) * (unsigned)sizeof(TH);
    const unsigned char* colB = reinterpret_cast<const unsigned char*>(H + col * Nz * (size_t)nt * 3);
    T dec = (T)1;
    if constexpr (!std::is_same<T, TH>::value) dec = (T)decode[0];
    const int ntile = (Nz + ZT - 1) / ZT;
    // the tile's ZT + 1 nodes k ZT + i; past node N_z - 1 they wrap (node N_z
    // is node 0), which only the last tile reaches
    auto wraps = [=](int k) { return k * ZT + ZT >= Nz; };
    auto node_off = [=](int k, int i) {
        const int z = k * ZT + i;
        return off0 + (unsigned)(z < Nz ? z : z % Nz) * zs_b;
    };
    auto load_tile = [=](RawTile<ZT, TH>& t, int k) {
        if (!wraps(k)) {
#pragma unroll
            for (int i = 0; i <= ZT; ++i) load_lag(colB, off0 + (unsigned)(k * ZT + i) * zs_b, t.n[i]);
        } else {
#pragma unroll
            for (int i = 0; i <= ZT; ++i) load_lag(colB, node_off(k, i), t.n[i]);
        }
    };
    // float16: the shift of node k ZT + i's lag in its loaded word; with ZT
    // even it only depends on the parity of i, except in the last tile
    const unsigned sh_even = (off0 & 2u) * 8u, sh_odd = ((off0 + zs_b) & 2u) * 8u;
    auto write_rows = [=](const RawTile<ZT, TH>& t, int k) {
        if (tid < nt) {
            // the lane's entry in row 0, made opaque so that the ZT + 1 row
            // addresses are added here rather than kept live across the loop
            int base = 64 + tid;
            asm volatile("" : "+v"(base));
            if (ZT % 2 == 0 && !wraps(k)) {
#pragma unroll
                for (int i = 0; i <= ZT; ++i) store_lag(t.n[i], (i & 1) ? sh_odd : sh_even, rows + base + i * RL);
            } else {
#pragma unroll
                for (int i = 0; i <= ZT; ++i) store_lag(t.n[i], (node_off(k, i) & 2u) * 8u, rows + base + i * RL);
            }
        }
    };
    auto zo = [=](int z) -> unsigned { return __builtin_amdgcn_readfirstlane(zoff[z < Nz ? z : Nz]); };
    // non-empty tiles, 64 at a time: bit i of msk is tile k0 + i
    auto scan_tiles = [=](int k) -> unsigned long long {
        const int t = k + lane;
        bool ne = false;
        if (t < ntile) ne = zoff[min(t * ZT + ZT, Nz)] != zoff[t * ZT];
        return __ballot(ne);
    };
    int k0 = 0;
    unsigned long long msk = 0;
    auto next_tile = [&scan_tiles, ntile](int k, int& k0, unsigned long long& msk) -> int {
        while (k < ntile) {
            if (k >= k0 + kWave) {
                k0 = k;
                msk = scan_tiles(k);
            }
            const unsigned long long rest = msk >> (k - k0);
            if (rest) return k + (int)__builtin_ctzll(rest);
            k = k0 + kWave;
        }
        return ntile;
    };
    __syncthreads();
    msk = scan_tiles(0);
    // LDS byte addresses: this lane's lag 0 in row 0, and row 0's first entry
    const unsigned rows_ab = (unsigned)(size_t)rows;
    const unsigned lane_ab = rows_ab + (unsigned)(64 + tid) * LB;
    typename SlotSums<T>::V acc = {};
    // the per-track sums to the output: one atomic per sample and track
    const int used = __popcll(__ballot(tabv >= 0));
    // (the lane test inside the loop: a branch on it around the loop would
    // join with the record loop's control flow and make that divergent)
    auto flush = [=](const typename SlotSums<T>::V& a) {
        for (int k = 0; k < used; ++k) {
            const int trk = __builtin_amdgcn_readlane(tabv, k);
            const T v = a[k];
            if (tid < nt && v != (T)0) atomicAdd(out + (size_t)trk * nt + tid, v * dec);
        }
    };
    unsigned since = 0, pf = 0;
    int k = next_tile(0, k0, msk);                       // there is one: the column has records
    RawTile<ZT, TH> nx;
    load_tile(nx, k);
    while (k < ntile) {
        __syncthreads();                                 // the previous tile's rows are read
        write_rows(nx, k);
        __syncthreads();
        const unsigned rbeg = zo(k * ZT), rend = zo(k * ZT + ZT);
        const int kn = next_tile(k + 1, k0, msk);
        if (kn < ntile) {
            load_tile(nx, kn);                           // lands while this tile is processed
            // the next tile's records pulled into the caches (a word of
            // every 64 bytes, up to 4 KB), so that its scalar reads hit
            asm volatile("" ::"v"(pf));                  // the previous pull has landed
            const unsigned a = zo(kn * ZT), b = zo(kn * ZT + ZT);
            const unsigned words = (b - a) * (unsigned)(sizeof(NodeRec<T>) / 4);
            const unsigned w = min((unsigned)lane * 16u, words - 1u);
            pf = reinterpret_cast<const unsigned*>(rec + cbeg + a)[w];
        }
        // the tile's records in groups that end where the sums are due out,
        // four at a time (their loads and LDS reads in flight together),
        // each added to its track's sum
        for (unsigned s0 = rbeg; s0 < rend;) {
            const unsigned s1 = min(s0 + (kFlushRecords - since), rend);
            const Const<NodeRec<T>>* q = crec + s0;
            for (; q + 4 <= crec + s1; q += 4) {
                const RecRegs<T> R0 = record_regs(q), R1 = record_regs(q + 1);
                const RecRegs<T> R2 = record_regs(q + 2), R3 = record_regs(q + 3);
                const T v0 = record_term<T, TH>(lane_ab, rows_ab, row_b, R0);
                const T v1 = record_term<T, TH>(lane_ab, rows_ab, row_b, R1);
                const T v2 = record_term<T, TH>(lane_ab, rows_ab, row_b, R2);
                const T v3 = record_term<T, TH>(lane_ab, rows_ab, row_b, R3);
                acc[(unsigned)R0.w1 >> 24] += v0;
                acc[(unsigned)R1.w1 >> 24] += v1;
                acc[(unsigned)R2.w1 >> 24] += v2;
                acc[(unsigned)R3.w1 >> 24] += v3;
            }
            for (; q != crec + s1; ++q) {
                const RecRegs<T> R = record_regs(q);
                acc[(unsigned)R.w1 >> 24] += record_term<T, TH>(lane_ab, rows_ab, row_b, R);
            }
            since += s1 - s0;
            s0 = s1;
            if (since >= kFlushRecords) {
                flush(acc);
                acc = typename SlotSums<T>::V{};
                since = 0;
            }
        }
        k = kn;
    }
    flush(acc);
}

// The overflow list: each wavefront takes runs of kOvfRun consecutive
// entries (a grid-stride loop over the count k_slots left), lanes over output
// samples n = lane + 64 j; each entry's two z-nodes are read from global
// memory at lag n - m and added to the lane's sums, which go to the output
// (one atomic per sample) when the track changes and at the end of the run.
// Entries of one column and chunk are consecutive in the list, so a run
// mostly holds few tracks.
template <typename T, typename TH>
__device__ inline T node_lag_dot(const Plan& p, const TH* colH, int z, int lag, const T* g) {
    const int TB = p.tb, nt = p.n_time, Nz = p.N[2];
    const int tb = lag / TB, tin = lag - tb * TB, nb = (nt + TB - 1) / TB;
    const int len = tb == nb - 1 ? nt - (nb - 1) * TB : TB;
    const TH* h = colH + (size_t)tb * TB * Nz * 3 + (size_t)z * len * 3 + tin * 3;
    return g[0] * (T)h[0] + g[1] * (T)h[1] + g[2] * (T)h[2];
}

template <typename T, typename TH>
__global__ void __launch_bounds__(kBlock)
k_conv_overflow(Plan p, const TH* __restrict__ H, const float* __restrict__ decode, const NodeRec<T>* rec,
                const unsigned long long* __restrict__ ctl, T* __restrict__ out) {
    if (ctl[kCtlFallback] != 0ull) return;
    const int lane = threadIdx.x & (kWave - 1);
    const unsigned long long n_ovf = ctl[kCtlOverflow];
    const OvfRec<T>* ovf = reinterpret_cast<const OvfRec<T>*>(rec + ((ctl[kCtlRecords] + 1) & ~1ull));
    const int nt = p.n_time, Nz = p.N[2];
    T dec = (T)1;
    if constexpr (!std::is_same<T, TH>::value) dec = (T)decode[0];
    const size_t waves = (size_t)gridDim.x * (kBlock / kWave);
    T acc[kMaxJ];
    auto flush = [&](int track) {
#pragma unroll
        for (int j = 0; j < kMaxJ; ++j) {
            const int n = lane + kWave * j;
            if (n < nt && acc[j] != (T)0) atomicAdd(out + (size_t)track * nt + n, acc[j] * dec);
            acc[j] = (T)0;
        }
    };
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) acc[j] = (T)0;
    for (size_t i0 = ((size_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * kOvfRun; i0 < n_ovf;
         i0 += waves * kOvfRun) {
        const size_t i1 = min(i0 + (size_t)kOvfRun, (size_t)n_ovf);
        int cur = ovf[i0].track;
        for (size_t i = i0; i < i1; ++i) {
            const OvfRec<T> o = ovf[i];
            if (o.track != cur) {
                flush(cur);
                cur = o.track;
            }
            const int m = o.zm & 0xffff, z0 = o.zm >> 16, z1 = z0 + 1 == Nz ? 0 : z0 + 1;
            const TH* colH = H + (size_t)o.col * Nz * nt * 3;
#pragma unroll
            for (int j = 0; j < kMaxJ; ++j) {
                const int n = lane + kWave * j;
                if (n >= m && n < nt)
                    acc[j] += node_lag_dot<T, TH>(p, colH, z0, n - m, o.g) +
                              node_lag_dot<T, TH>(p, colH, z1, n - m, o.g + 3);
            }
        }
        flush(cur);
    }
}

// phase 1: the output zeroed and the events binned; phase 2: the
// accumulation (binned, or the unbinned kernel when the events did not fit
// or there is no workspace).  Phase 2 follows phase 1 on the same stream.
// Phase 2 split in two for two streams: phase 4 is the accumulation without
// the overflow list, phase 3 the overflow list alone (nothing when the form
// is not binned); both only add into the output, so they may run at once.
// max_blocks > 0 caps the grids of the per-carrier and per-column binning
// kernels (their wavefronts stride over the work).
template <typename T, typename TH>
hipError_t current(const Plan& p, const void* h, int n_carriers, int n_tracks, const void* pos, const void* charge,
                   const int* track, void* ws, size_t ws_bytes, void* out, hipStream_t s, int phase, int form,
                   int max_blocks) {
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
    const ConvTiling tl = conv_tiling(p);
    const CurrentLayout cl = current_layout(p, tl, n_carriers);
    static_assert(sizeof(NodeRec<float>) == 32 && sizeof(NodeRec<double>) == 64, "record size");
    // per-cell counts are 32-bit: bin only while every step fits them; below
    // kBinnedMinSteps polyline steps the unbinned kernel is faster (its cost
    // is the steps that move, the binned form's also the grid's columns)
    const unsigned long long steps = (unsigned long long)n_carriers * p.n_time;
    const bool binned = ws != nullptr && ws_bytes >= cl.fixed_bytes + 4 * sizeof(NodeRec<T>) && steps < 0xfffffff0ull &&
                        form != 2 && (steps >= kBinnedMinSteps || form == 1);
    unsigned long long* ctl = nullptr;
    if (binned) {
        char* b = static_cast<char*>(ws);
        ctl = reinterpret_cast<unsigned long long*>(b + cl.off_ctl);
        unsigned* count = reinterpret_cast<unsigned*>(b + cl.off_count);
        unsigned* fill = reinterpret_cast<unsigned*>(b + cl.off_fill);
        unsigned* offs = reinterpret_cast<unsigned*>(b + cl.off_offs);
        unsigned long long* bsum = reinterpret_cast<unsigned long long*>(b + cl.off_bsum);
        uint4* base = reinterpret_cast<uint4*>(b + cl.off_base);
        unsigned long long* mask = reinterpret_cast<unsigned long long*>(b + cl.off_mask);
        int* tables = reinterpret_cast<int*>(b + cl.off_tables);
        NodeRec<T>* rec = reinterpret_cast<NodeRec<T>*>(b + cl.off_records);
        size_t cap = (ws_bytes - cl.off_records) / sizeof(NodeRec<T>);
        if (cap > 0xfffffff0ull) cap = 0xfffffff0ull;
        if (phase == 1) {
            // control words, cell counts and fill counters are one zero-filled
            // run (no memset nodes, so the sequence can be captured)
            auto capped = [&](size_t g) {
                return (unsigned)(max_blocks > 0 && g > (size_t)max_blocks ? (size_t)max_blocks : g);
            };
            const size_t n_zero = cl.off_offs / sizeof(unsigned);
            hipLaunchKernelGGL(k_fill_zero<unsigned>,
                               dim3(capped(std::min<size_t>((n_zero + kBlock - 1) / kBlock, 4096))), dim3(kBlock),
                               0, s, reinterpret_cast<unsigned*>(b), n_zero);
            hipLaunchKernelGGL(k_set_capacity, dim3(1), dim3(1), 0, s, ctl, (unsigned long long)cap);
            const unsigned grid = capped(((size_t)n_carriers + kBlock / kWave - 1) / (kBlock / kWave));
            hipLaunchKernelGGL(k_ev_count<T>, dim3(grid), dim3(kBlock), 0, s, p, tl, n_carriers, n_tracks,
                               static_cast<const T*>(pos), track, mask, count);
            const unsigned cell_grid = capped(std::min<size_t>((tl.n_cells + kBlock - 1) / kBlock, 65536));
            hipLaunchKernelGGL(k_node_count, dim3(cell_grid), dim3(kBlock), 0, s, p, count, offs);
            const unsigned nb = (unsigned)((tl.n_cells + kScanItems - 1) / kScanItems);
            hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, s, offs, tl.n_cells, bsum);
            hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, bsum, (int)nb, ctl);
            hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, s, offs, tl.n_cells, bsum);
            hipLaunchKernelGGL(k_cell_bases, dim3(cell_grid), dim3(kBlock), 0, s, p, count, offs, base);
            hipLaunchKernelGGL(k_ev_scatter<T>, dim3(grid), dim3(kBlock), 0, s, p, tl, n_carriers,
                               static_cast<const T*>(pos), static_cast<const T*>(charge), track, mask, fill, base,
                               ctl, rec);
            const size_t slots_grid = (tl.n_cols + kBlock / kWave - 1) / (kBlock / kWave);
            if (capped(slots_grid) < slots_grid)
                hipLaunchKernelGGL((k_slots<T, true>), dim3(capped(slots_grid)), dim3(kBlock), 0, s, p, tl, offs, rec,
                                   ctl, tables);
            else
                hipLaunchKernelGGL((k_slots<T, false>), dim3(slots_grid), dim3(kBlock), 0, s, p, tl, offs, rec, ctl,
                                   tables);
            return hipGetLastError();
        }
        auto rows = [&](auto kernel) {
            e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)tl.lds_bytes);
            if (e != hipSuccess) return;
            hipLaunchKernelGGL(kernel, dim3((unsigned)tl.n_cols), dim3(tl.threads), tl.lds_bytes, s, p, tl,
                               static_cast<const TH*>(h), decode, offs, rec, tables, ctl,
                               static_cast<T*>(out));
        };
        if (phase != 3) {
            // tiles of conv_tile_nodes(sizeof(TH)) z-nodes
            rows(k_conv_rows<conv_tile_nodes(sizeof(TH)), T, TH>);
            if (e != hipSuccess) return e;
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        if (phase != 4) {
            hipLaunchKernelGGL((k_conv_overflow<T, TH>), dim3(1024), dim3(kBlock), 0, s, p,
                               static_cast<const TH*>(h), decode, rec, ctl, static_cast<T*>(out));
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (phase == 1 || phase == 3) return hipSuccess;
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
                          hipStream_t s, int phase, int form, int max_blocks) {
    if (p.precision == 0)
        return current<double, double>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s, phase,
                                       form, max_blocks);
    if (p.h_format == 1)
        return current<float, _Float16>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s, phase,
                                        form, max_blocks);
    return current<float, float>(p, h, n_carriers, n_tracks, pos, charge, track, ws, ws_bytes, out, s, phase, form,
                                 max_blocks);
}

}  // namespace wt
