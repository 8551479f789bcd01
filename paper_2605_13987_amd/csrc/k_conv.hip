// Induced current, Eq. 1 of the paper (introduction):
//   i(t) = -(q / V_w) int_0^t H(x(t'), t - t') . v(t') dt',  V_w = 1 V,
// discretised on the time grid: every polyline step m of a carrier with a
// non-zero displacement dx contributes, at every later sample n >= m, the
// field at the step midpoint and lag n - m projected on dx; the field between
// nodes is the trilinear interpolation of the nodal H with periodic wrap.
// Section 3 of the paper computes the whole correlation of one carrier per
// GPU thread; here one 64-lane wavefront owns a few carriers and its lanes
// own output samples n = lane + 64 j, so the 8 corner lag series of a step
// are read as contiguous runs and the sum over steps stays in registers.
#include "common.hpp"

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

template <typename T>
__global__ void __launch_bounds__(kBlock)
k_current(Plan p, const T* H, int n_carriers, int n_tracks, const T* pos, const T* charge,
          const int* track, T* out, int per_wave) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave);
    const int c_begin = wave * per_wave;
    const int c_end = min(c_begin + per_wave, n_carriers);
    const int nt = p.n_time, TB = p.tb;
    const int Nx = p.N[0], Ny = p.N[1], Nz = p.N[2];
    const int last_block = (nt - 1) / TB;
    const int last_len = nt - last_block * TB;
    const size_t col_stride = (size_t)Nz * nt * 3;
    const T ihx = (T)(Nx / p.L[0]), ihy = (T)(Ny / p.L[1]), ihz = (T)(Nz / p.L[2]);

    T acc[kMaxJ];
#pragma unroll
    for (int j = 0; j < kMaxJ; ++j) acc[j] = (T)0;
    int cur = -1;

    for (int c = c_begin; c < c_end; ++c) {
        const int tr = track[c];
        if (tr < 0 || tr >= n_tracks) continue;
        if (tr != cur) {
            if (cur >= 0) flush(out, cur, nt, lane, acc);
            cur = tr;
        }
        const T q = charge[c];
        const T* P = pos + (size_t)c * (nt + 1) * 3;
        for (int m = 0; m < nt; ++m) {
            const T dx = P[3 * m + 3] - P[3 * m + 0];
            const T dy = P[3 * m + 4] - P[3 * m + 1];
            const T dz = P[3 * m + 5] - P[3 * m + 2];
            if (dx == (T)0 && dy == (T)0 && dz == (T)0) continue;
            const T ux = (P[3 * m + 0] + P[3 * m + 3]) * (T)0.5 * ihx;
            const T uy = (P[3 * m + 1] + P[3 * m + 4]) * (T)0.5 * ihy;
            const T uz = (P[3 * m + 2] + P[3 * m + 5]) * (T)0.5 * ihz;
            if (!(isfinite(ux) && isfinite(uy) && isfinite(uz))) continue;
            const T flx = floor(ux), fly = floor(uy), flz = floor(uz);
            const T fx = ux - flx, fy = uy - fly, fz = uz - flz;
            // periodic wrap of the lower corner, clamped so every index is in range
            const int x0 = wrap_index(flx, Nx), y0 = wrap_index(fly, Ny), z0 = wrap_index(flz, Nz);
            const int x1 = x0 + 1 == Nx ? 0 : x0 + 1;
            const int y1 = y0 + 1 == Ny ? 0 : y0 + 1;
            const int z1 = z0 + 1 == Nz ? 0 : z0 + 1;
            const size_t b00 = ((size_t)x0 * Ny + y0) * col_stride, b01 = ((size_t)x0 * Ny + y1) * col_stride;
            const size_t b10 = ((size_t)x1 * Ny + y0) * col_stride, b11 = ((size_t)x1 * Ny + y1) * col_stride;
            const T gx0 = (T)1 - fx, gy0 = (T)1 - fy, gz0 = (T)1 - fz;
            // -q folded into the weights (V_w = 1 V)
            const T w000 = -q * gx0 * gy0 * gz0, w001 = -q * gx0 * gy0 * fz;
            const T w010 = -q * gx0 * fy * gz0, w011 = -q * gx0 * fy * fz;
            const T w100 = -q * fx * gy0 * gz0, w101 = -q * fx * gy0 * fz;
            const T w110 = -q * fx * fy * gz0, w111 = -q * fx * fy * fz;
#pragma unroll
            for (int j = 0; j < kMaxJ; ++j) {
                const int n = lane + kWave * j;
                const int tau = n - m;
                if (n >= nt || tau < 0) continue;
                const int tb = tau / TB;
                const int tin = tau - tb * TB;
                const int len = tb == last_block ? last_len : TB;
                const size_t toff = (size_t)tb * TB * Nz * 3 + (size_t)tin * 3;
                const size_t o0 = toff + (size_t)z0 * len * 3, o1 = toff + (size_t)z1 * len * 3;
                const T* h;
                T v = (T)0;
                h = H + b00 + o0; v += w000 * (h[0] * dx + h[1] * dy + h[2] * dz);
                h = H + b00 + o1; v += w001 * (h[0] * dx + h[1] * dy + h[2] * dz);
                h = H + b01 + o0; v += w010 * (h[0] * dx + h[1] * dy + h[2] * dz);
                h = H + b01 + o1; v += w011 * (h[0] * dx + h[1] * dy + h[2] * dz);
                h = H + b10 + o0; v += w100 * (h[0] * dx + h[1] * dy + h[2] * dz);
                h = H + b10 + o1; v += w101 * (h[0] * dx + h[1] * dy + h[2] * dz);
                h = H + b11 + o0; v += w110 * (h[0] * dx + h[1] * dy + h[2] * dz);
                h = H + b11 + o1; v += w111 * (h[0] * dx + h[1] * dy + h[2] * dz);
                acc[j] += v;
            }
        }
    }
    if (cur >= 0) flush(out, cur, nt, lane, acc);
}

template <typename T>
hipError_t current(const Plan& p, const void* h, int n_carriers, int n_tracks, const void* pos,
                   const void* charge, const int* track, void* out, hipStream_t s) {
    const size_t n_out = (size_t)n_tracks * p.n_time;
    const int zgrid = (int)((n_out + kBlock - 1) / kBlock < 4096 ? (n_out + kBlock - 1) / kBlock : 4096);
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(zgrid > 0 ? zgrid : 1), dim3(kBlock), 0, s, static_cast<T*>(out), n_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_carriers == 0) return e;
    const int per_wave = 4;
    const int waves = (n_carriers + per_wave - 1) / per_wave;
    const int blocks = (waves * kWave + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_current<T>, dim3(blocks), dim3(kBlock), 0, s, p, static_cast<const T*>(h), n_carriers,
                       n_tracks, static_cast<const T*>(pos), static_cast<const T*>(charge), track,
                       static_cast<T*>(out), per_wave);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_current(const Plan& p, const void* h, int n_carriers, int n_tracks, const void* pos,
                          const void* charge, const int* track, void* out, hipStream_t s) {
    return p.precision == 0 ? current<double>(p, h, n_carriers, n_tracks, pos, charge, track, out, s)
                            : current<float>(p, h, n_carriers, n_tracks, pos, charge, track, out, s);
}

}  // namespace wt
