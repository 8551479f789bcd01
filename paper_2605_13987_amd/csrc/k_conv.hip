// Induced current, Eq. 1 of the paper (introduction):
//   i(t) = -(q / V_w) int_0^t H(x(t'), t - t') . v(t') dt',  V_w = 1 V,
// discretised on the time grid: every polyline step m of a carrier with a
// non-zero displacement dx contributes, at every later sample n >= m, the
// field at the step midpoint and lag n - m projected on dx; the field between
// nodes is the trilinear interpolation of the nodal H with periodic wrap.
// Section 3 of the paper computes the whole correlation of one carrier per
// GPU thread; here one 64-lane wavefront owns a carrier and its lanes own
// output samples n = lane + 64 j, so the 8 corner lag series of a step are
// read as contiguous runs and the sum over steps stays in registers.
#include "common.hpp"

#include <type_traits>

namespace wt {

namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kMaxJ = kMaxTime / kWave;

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
    const int Nx = p.N[0], Ny = p.N[1], Nz = p.N[2];
    const size_t col_stride = (size_t)Nz * p.n_time * 3;
    s.dx = P[3 * m + 3] - P[3 * m + 0];
    s.dy = P[3 * m + 4] - P[3 * m + 1];
    s.dz = P[3 * m + 5] - P[3 * m + 2];
    const T ux = (P[3 * m + 0] + P[3 * m + 3]) * (T)0.5 * (T)(Nx / p.L[0]);
    const T uy = (P[3 * m + 1] + P[3 * m + 4]) * (T)0.5 * (T)(Ny / p.L[1]);
    const T uz = (P[3 * m + 2] + P[3 * m + 5]) * (T)0.5 * (T)(Nz / p.L[2]);
    if (!(isfinite(ux) && isfinite(uy) && isfinite(uz))) return false;
    const T flx = floor(ux), fly = floor(uy), flz = floor(uz);
    const T fx = ux - flx, fy = uy - fly, fz = uz - flz;
    // periodic wrap of the lower corner, clamped so every index is in range
    const int x0 = wrap_index(flx, Nx), y0 = wrap_index(fly, Ny), z0 = wrap_index(flz, Nz);
    const int x1 = x0 + 1 == Nx ? 0 : x0 + 1;
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
// once per output sample.  Neighbouring carriers read neighbouring corners,
// and those reads are shared through the caches only while the carriers are
// processed at the same time: workgroups are dealt to the 8 XCDs round robin,
// so carriers are numbered such that the workgroups resident on one XCD hold
// consecutive carriers, whose common reads its L2 then serves.
template <int TBC, typename T, typename TH>
__global__ void __launch_bounds__(kBlock)
k_current(Plan p, const TH* H, const float* decode, int n_carriers, int n_tracks, const T* pos, const T* charge,
          const int* track, T* out) {
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

template <typename T, typename TH>
hipError_t current(const Plan& p, const void* h, int n_carriers, int n_tracks, const void* pos,
                   const void* charge, const int* track, void* out, hipStream_t s) {
    const size_t n_out = (size_t)n_tracks * p.n_time;
    const int zgrid = (int)((n_out + kBlock - 1) / kBlock < 4096 ? (n_out + kBlock - 1) / kBlock : 4096);
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(zgrid > 0 ? zgrid : 1), dim3(kBlock), 0, s, static_cast<T*>(out), n_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_carriers == 0) return e;
    // the carriers of workgroup b come from a permutation of [0, 8 * per_xcd)
    // workgroups (some past the last carrier, which then do nothing)
    const int blocks = (n_carriers + kBlock / kWave - 1) / (kBlock / kWave);
    const int grid = 8 * ((blocks + 7) / 8);
    const float* decode = reinterpret_cast<const float*>(static_cast<const char*>(h) + p.h_values_bytes);
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, s, p, static_cast<const TH*>(h), decode, n_carriers,
                           n_tracks, static_cast<const T*>(pos), static_cast<const T*>(charge), track,
                           static_cast<T*>(out));
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
                          const void* charge, const int* track, void* out, hipStream_t s) {
    if (p.precision == 0) return current<double, double>(p, h, n_carriers, n_tracks, pos, charge, track, out, s);
    if (p.h_format == 1) return current<float, _Float16>(p, h, n_carriers, n_tracks, pos, charge, track, out, s);
    return current<float, float>(p, h, n_carriers, n_tracks, pos, charge, track, out, s);
}

}  // namespace wt
