// Spectral extension of the boundary solution to the bulk (paper, abstract:
// spectral methods extend the solution to the bulk; Section 3: spectra are
// multiplied by the wave-vector terms in a custom kernel).
//
// H(x, t_n) = sum_k M(k) exp(i k.x) sum_i q_i(t_n) exp(-i k.y_i) over the grid's
// modes (|m_a| < N_a/2, k != 0), with
//   M(k) = -i k S(k) / (eps |k|^2 V),  S(k) = exp(-sum_a k_a^2 s_a^2 / 2).
// Every source sits on a column axis (X_w, Y_w) on a grid node, so the sum
// factors into an in-plane table, built once per geometry,
//   Ehat_a(X, Y, m_z) = sum_{m_x, m_y} M_a(k) exp(i (k_x X + k_y Y))
// (a 2D inverse FFT per (m_z, a)), and a per-column synthesis along z,
//   H_a(X, Y, z, t) = sum_{m_z} exp(i k_z z) sum_w Ehat_a(X - X_w, Y - Y_w, m_z) Qhat_w(m_z, t),
// a Hermitian (complex-to-real) inverse FFT of length N_z per (X, Y, t, a).
// Two real outputs share one complex FFT: Z = F_1 + i F_2, Re -> 1, Im -> 2.
#include "synth_pipe.hpp"

#include <algorithm>
#include <type_traits>

namespace wt {

namespace {

constexpr int kBlock = 256;
// LDS of one line-FFT block (two buffers): 32 KB lets four blocks share a CU;
// at 256 x 256 x 512 the field table took 1.13 ms against 1.45 ms with 64 KB
// (two blocks per CU) and 1.29 ms with 16 KB.
constexpr size_t kLineLds = 32 * 1024;

// deriv = 1: the derivative of M(k) under a uniform scaling of the cell's
// in-plane size (pitch) by s, at s = 1, with the grid counts held: k_x and
// k_y scale as 1/s, k_x s_x and k_y s_y are unchanged and V scales as s^2, so
// dM_a/ds = M_a (2 (k_x^2 + k_y^2)/|k|^2 - 2 - [a in {x, y}]).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_multiplier(Plan p, int deriv, cplx<T>* e) {
    const int Nx = p.N[0], Ny = p.N[1], nzh = p.nzh;
    const size_t total = (size_t)Nx * Ny * nzh;
    const double vol = p.L[0] * p.L[1] * p.L[2];
    for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (size_t)gridDim.x * blockDim.x) {
        const int mz = (int)(idx % nzh);
        const int iy = (int)((idx / nzh) % Ny);
        const int ix = (int)(idx / ((size_t)nzh * Ny));
        const int mx = ix < Nx / 2 ? ix : ix - Nx;
        const int my = iy < Ny / 2 ? iy : iy - Ny;
        cplx<T>* out = e + idx * 3;
        if (ix == Nx / 2 || iy == Ny / 2 || (mx == 0 && my == 0 && mz == 0)) {
            out[0] = out[1] = out[2] = cplx<T>{(T)0, (T)0};
            continue;
        }
        const double kx = 2.0 * kPi * mx / p.L[0];
        const double ky = 2.0 * kPi * my / p.L[1];
        const double kz = 2.0 * kPi * mz / p.L[2];
        const double k2 = kx * kx + ky * ky + kz * kz;
        const double ax = kx * p.s_bulk[0], ay = ky * p.s_bulk[1], az = kz * p.s_bulk[2];
        const double w = exp(-0.5 * (ax * ax + ay * ay + az * az)) / (k2 * p.eps * vol);
        const double d = deriv ? 2.0 * (kx * kx + ky * ky) / k2 - 2.0 : 1.0;
        const double dxy = deriv ? d - 1.0 : 1.0;
        out[0] = cplx<T>{(T)0, (T)(-kx * w * dxy)};
        out[1] = cplx<T>{(T)0, (T)(-ky * w * dxy)};
        out[2] = cplx<T>{(T)0, (T)(-kz * w * d)};
    }
}

// In-place inverse FFTs along one grid axis of a strided array.  Line l has
// its first element at (l / n_inner) * outer_stride + (l % n_inner) and its
// elements elem_stride apart; a block transforms lpb lines with consecutive
// inner index so that loads and stores touch contiguous runs.  NC: the
// line length when it is a power of two fixed at compile time, else 0.
template <typename T, int NC>
__global__ void __launch_bounds__(kBlock)
k_fft_lines(Plan p, int axis, cplx<T>* data, int n_inner, int n_lines, size_t outer_stride,
            size_t elem_stride, int lpb, const cplx<T>* tw) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int N = NC > 0 ? NC : p.N[axis];
    cplx<T>* a = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* b = a + (size_t)lpb * N;
    const int l0 = blockIdx.x * lpb;
    const int nl = min(lpb, n_lines - l0);
    for (int idx = threadIdx.x; idx < nl * N; idx += blockDim.x) {
        const int e = idx / nl, f = idx - e * nl;
        const int l = l0 + f;
        const size_t base = (size_t)(l / n_inner) * outer_stride + (size_t)(l % n_inner);
        a[f * N + e] = data[base + e * elem_stride];
    }
    __syncthreads();
    const cplx<T>* res;
    if constexpr (NC > 0)
        res = fft_inverse_lds_pow2<T, NC>(a, b, nl, tw);
    else
        res = fft_inverse_lds<T>(a, b, N, nl, p.rad[axis], p.nrad[axis], tw);
    for (int idx = threadIdx.x; idx < nl * N; idx += blockDim.x) {
        const int e = idx / nl, f = idx - e * nl;
        const int l = l0 + f;
        const size_t base = (size_t)(l / n_inner) * outer_stride + (size_t)(l % n_inner);
        data[base + e * elem_stride] = res[f * N + e];
    }
}

// Spectrum of real signal s (= 3 * time-in-block + component) at z-frequency
// index k in [0, N_z): F(k) for k < N_z/2, conj(F(N_z - k)) above, 0 at N_z/2.
template <typename T>
__device__ inline cplx<T> column_spectrum(const Plan& p, const cplx<T>* etab, const cplx<T>* qhat,
                                          int t0, int nsig, int s, int k) {
    const int nzh = p.nzh;
    if (s >= nsig || k == nzh) return cplx<T>{(T)0, (T)0};
    const int t = t0 + s / 3, a = s % 3;
    const bool upper = k > nzh;
    const int kk = upper ? p.N[2] - k : k;
    cplx<T> acc{(T)0, (T)0};
    const cplx<T>* q = qhat + (size_t)t * p.n_cols * nzh + kk;
    for (int w = 0; w < p.n_cols; ++w) acc = acc + etab[(w * nzh + kk) * 3 + a] * q[(size_t)w * nzh];
    return upper ? conj(acc) : acc;
}

// One block per (X, Y) column: H for every z node and time sample, written
// one time block at a time as a contiguous run [z][t in block][component].
constexpr int kSynthMaxBlock = 1024;

template <typename T>
__global__ void __launch_bounds__(kSynthMaxBlock)
k_synthesis(Plan p, const cplx<T>* ehat, const cplx<T>* qhat, const cplx<T>* tw, T* H, int fb) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int Nx = p.N[0], Ny = p.N[1], Nz = p.N[2], nzh = p.nzh, W = p.n_cols;
    const int nt = p.n_time, TB = p.tb;
    cplx<T>* etab = reinterpret_cast<cplx<T>*>(smem);
    cplx<T>* fa = etab + W * nzh * 3;
    cplx<T>* fbuf = fa + (size_t)fb * Nz;
    T* stage = reinterpret_cast<T*>(fbuf + (size_t)fb * Nz);

    const int col = blockIdx.x;
    const int ix = col / Ny, iy = col - (col / Ny) * Ny;
    for (int idx = threadIdx.x; idx < W * nzh * 3; idx += blockDim.x) {
        const int w = idx / (nzh * 3), r = idx - w * (nzh * 3);
        const int sx = (ix - p.col[w].ix + Nx) % Nx;
        const int sy = (iy - p.col[w].iy + Ny) % Ny;
        etab[idx] = ehat[((size_t)sx * Ny + sy) * nzh * 3 + r];
    }
    __syncthreads();

    T* hcol = H + (size_t)col * Nz * nt * 3;
    for (int t0 = 0; t0 < nt; t0 += TB) {
        const int tbl = min(TB, nt - t0);
        const int nsig = 3 * tbl;
        const int npair = (nsig + 1) / 2;
        for (int pb = 0; pb < npair; pb += fb) {
            const int nf = min(fb, npair - pb);
            for (int idx = threadIdx.x; idx < nf * Nz; idx += blockDim.x) {
                const int f = idx / Nz, k = idx - f * Nz;
                const int s0 = 2 * (pb + f);
                const cplx<T> z0 = column_spectrum<T>(p, etab, qhat, t0, nsig, s0, k);
                const cplx<T> z1 = column_spectrum<T>(p, etab, qhat, t0, nsig, s0 + 1, k);
                fa[idx] = z0 + mul_i(z1);
            }
            __syncthreads();
            const cplx<T>* res = fft_inverse_lds<T>(fa, fbuf, Nz, nf, p.rad[2], p.nrad[2], tw);
            for (int idx = threadIdx.x; idx < nf * Nz; idx += blockDim.x) {
                const int f = idx / Nz, z = idx - f * Nz;
                const int s0 = 2 * (pb + f);
                const cplx<T> v = res[idx];
                stage[(z * tbl + s0 / 3) * 3 + s0 % 3] = v.re;
                if (s0 + 1 < nsig) stage[(z * tbl + (s0 + 1) / 3) * 3 + (s0 + 1) % 3] = v.im;
            }
            __syncthreads();
        }
        T* dst = hcol + (size_t)t0 * Nz * 3;
        for (int idx = threadIdx.x; idx < Nz * nsig; idx += blockDim.x) dst[idx] = stage[idx];
        __syncthreads();
    }
}

// Scale of float16 H (stored value = H * h_scale).  H_a(X, Y, z, t) is the
// sum over k_z in (-N_z/2, N_z/2) of e^{i k_z z} sum_w Ehat_a(X - X_w,
// Y - Y_w, k_z) Qhat_w(k_z, t) (negative k_z as conjugates), so
//   |H| <= B = sum_{k >= 0} m_k max_{X,Y,a} |Ehat_a(X,Y,k)| sum_w max_t |Qhat_w(k,t)|
// with m_0 = 1 and m_k = 2 otherwise.  h_scale = 2^s with s the largest
// integer such that B h_scale <= 16384, a quarter of the float16 range: a
// power of two, so that scaling and unscaling are exact.
//
// k_hscale_emax: max over (X, Y, a) of |Ehat| per k_z, as the bits of a
// non-negative float (their integer order is the float order).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_hscale_emax(Plan p, const cplx<T>* ehat, unsigned* emax) {
    // the block size, and so the grid stride, is a multiple of N_z/2, so each
    // thread stays on one k_z; threads of a block with the same k_z combine
    // in LDS before one atomic per k_z
    __shared__ float m_lds[kBlock];
    const size_t n = (size_t)p.N[0] * p.N[1] * p.nzh;
    float m = 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const cplx<T>* e = ehat + i * 3;
#pragma unroll
        for (int a = 0; a < 3; ++a) m = fmaxf(m, (float)sqrt(e[a].re * e[a].re + e[a].im * e[a].im));
    }
    m_lds[threadIdx.x] = m;
    __syncthreads();
    if ((int)threadIdx.x < p.nzh) {
        for (int j = threadIdx.x + p.nzh; j < (int)blockDim.x; j += p.nzh) m = fmaxf(m, m_lds[j]);
        atomicMax(emax + threadIdx.x, __float_as_uint(m));
    }
}

__global__ void __launch_bounds__(kBlock) k_hscale_clear(unsigned* emax, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) emax[i] = 0u;
}

// One workgroup per k_z: qsum[k] = sum_w max_t |Qhat_w(k, t)|.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_hscale_qmax(Plan p, const cplx<T>* qhat, float* qsum) {
    __shared__ float part[kBlock];
    const int k = blockIdx.x, nzh = p.nzh, W = p.n_cols, nt = p.n_time;
    float acc = 0.0f;
    for (int w = 0; w < W; ++w) {
        float m = 0.0f;
        for (int t = threadIdx.x; t < nt; t += blockDim.x) {
            const cplx<T> q = qhat[((size_t)t * W + w) * nzh + k];
            m = fmaxf(m, (float)sqrt(q.re * q.re + q.im * q.im));
        }
        part[threadIdx.x] = m;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) part[threadIdx.x] = fmaxf(part[threadIdx.x], part[threadIdx.x + h]);
            __syncthreads();
        }
        acc += part[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) qsum[k] = acc;
}

// One workgroup: the bound B, then h_scale (workspace) and 1/h_scale (the
// float after the values of H).
__global__ void __launch_bounds__(kBlock)
k_hscale_finish(int nzh, const unsigned* emax, const float* qsum, float* scale, float* decode) {
    __shared__ double part[kBlock];
    double b = 0.0;
    for (int k = threadIdx.x; k < nzh; k += blockDim.x)
        b += (k == 0 ? 1.0 : 2.0) * (double)__uint_as_float(emax[k]) * (double)qsum[k];
    part[threadIdx.x] = b;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double B = part[0];
        int sc = 0;
        if (B > 0.0 && isfinite(B)) {
            sc = (int)floor(log2(16384.0 / B));
            while (ldexp(B, sc) > 16384.0) --sc;          // guard the rounding of log2
            sc = sc < -120 ? -120 : (sc > 120 ? 120 : sc);
        }
        scale[0] = ldexpf(1.0f, sc);
        decode[0] = ldexpf(1.0f, -sc);
    }
}

template <typename T>
int lines_per_block(int N) {
    int lpb = 64;
    while (lpb > 1 && (size_t)2 * lpb * N * sizeof(cplx<T>) > kLineLds) lpb >>= 1;
    return lpb;
}

// The field table (deriv = 0) or its pitch derivative (deriv = 1) into e.
template <typename T>
hipError_t field_table(const Plan& p, char* b, cplx<T>* e, int deriv, hipStream_t s) {
    const size_t total = (size_t)p.N[0] * p.N[1] * p.nzh;
    const int grid = (int)((total + kBlock - 1) / kBlock < 65536 ? (total + kBlock - 1) / kBlock : 65536);
    hipLaunchKernelGGL(k_multiplier<T>, dim3(grid), dim3(kBlock), 0, s, p, deriv, e);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    const int C = p.nzh * 3;
    for (int axis = 1; axis >= 0; --axis) {
        const int N = p.N[axis];
        const int lpb = lines_per_block<T>(N);
        const size_t lds = (size_t)2 * lpb * N * sizeof(cplx<T>);
        int n_lines;
        size_t outer, elem;
        if (axis == 1) {          // along y: lines (x, c)
            n_lines = p.N[0] * C;
            outer = (size_t)p.N[1] * C;
            elem = C;
        } else {                  // along x: lines (y, c)
            n_lines = p.N[1] * C;
            outer = C;
            elem = (size_t)p.N[1] * C;
        }
        const cplx<T>* tw = reinterpret_cast<const cplx<T>*>(b + p.off_tw[axis]);
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, dim3((n_lines + lpb - 1) / lpb), dim3(kBlock), lds, s, p, axis, e, C,
                               n_lines, outer, elem, lpb, tw);
        };
        switch (N) {
            case 64: go(k_fft_lines<T, 64>); break;
            case 128: go(k_fft_lines<T, 128>); break;
            case 256: go(k_fft_lines<T, 256>); break;
            case 512: go(k_fft_lines<T, 512>); break;
            default: go(k_fft_lines<T, 0>); break;
        }
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}


template <typename T, int N1, int N2, typename TO, int TB>
hipError_t synthesis_pipe_w(const Plan& p, char* b, void* h, hipStream_t s) {
    switch (p.n_cols) {
        case 1: return synthesis_pipe<T, N1, N2, 1, TO, TB>(p, b, h, s);
        case 2: return synthesis_pipe<T, N1, N2, 2, TO, TB>(p, b, h, s);
        case 3: return synthesis_pipe<T, N1, N2, 3, TO, TB>(p, b, h, s);
        default: return synthesis_pipe<T, N1, N2, 4, TO, TB>(p, b, h, s);
    }
}

// The power-of-two schedule I of kPow2Schedules that the plan names, if it
// fits in LDS for T.
template <int I, typename T, typename TO>
hipError_t synthesis_pipe_pow2(const Plan& p, char* b, void* h, hipStream_t s) {
    if constexpr (I == kNumPow2Schedules) {
        return hipErrorInvalidValue;
    } else {
        constexpr PipeSchedule c = kPow2Schedules[I];
        if constexpr (pipe_fits(pipe_shape_for(c.nz, c.n1, c.tbc), (int)sizeof(T))) {
            if (p.N[2] == c.nz && p.synth_n1 == c.n1 && p.synth_tbc == c.tbc)
                return synthesis_pipe_w<T, c.n1, c.nz / c.n1, TO, c.tbc>(p, b, h, s);
        }
        return synthesis_pipe_pow2<I + 1, T, TO>(p, b, h, s);
    }
}

template <typename T, typename TO>
hipError_t synthesis_pipe_n(const Plan& p, char* b, void* h, hipStream_t s) {
    if (!synthesis_pow2(p.N[2])) return launch_synthesis_smooth(p, b, h, s);
    return synthesis_pipe_pow2<0, T, TO>(p, b, h, s);
}

template <typename T>
hipError_t synthesis(const Plan& p, char* b, void* h, hipStream_t s) {
    if (p.synth_kernel == 2) {
        if constexpr (std::is_same<T, float>::value)
            if (p.h_format == 1) return synthesis_pipe_n<T, _Float16>(p, b, h, s);
        return synthesis_pipe_n<T, T>(p, b, h, s);
    }
    // fb sample-pair transforms per pass: all pairs of a block when they fit
    const size_t fixed = (size_t)p.n_cols * p.nzh * 3 * sizeof(cplx<T>) + (size_t)p.N[2] * p.tb * 3 * sizeof(T);
    const size_t budget = 160 * 1024;
    int fb = (3 * p.tb + 1) / 2;
    while (fb > 1 && fixed + (size_t)2 * fb * p.N[2] * sizeof(cplx<T>) > budget) --fb;
    const size_t lds = fixed + (size_t)2 * fb * p.N[2] * sizeof(cplx<T>);
    hipError_t err = hipFuncSetAttribute((const void*)k_synthesis<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)lds);
    if (err != hipSuccess) return err;
    if (p.synth_threads < 64 || p.synth_threads > kSynthMaxBlock || p.synth_threads % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_synthesis<T>, dim3(p.N[0] * p.N[1]), dim3(p.synth_threads), lds, s, p,
                       reinterpret_cast<const cplx<T>*>(b + p.off_ehat),
                       reinterpret_cast<const cplx<T>*>(b + p.off_qhat),
                       reinterpret_cast<const cplx<T>*>(b + p.off_tw[2]), static_cast<T*>(h), fb);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_field_table(const Plan& p, void* ws, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    return p.precision == 0 ? field_table<double>(p, b, reinterpret_cast<cplx<double>*>(b + p.off_ehat), 0, s)
                            : field_table<float>(p, b, reinterpret_cast<cplx<float>*>(b + p.off_ehat), 0, s);
}

hipError_t launch_field_table_pitch_derivative(const Plan& p, const void* ws, void* out, hipStream_t s) {
    char* b = const_cast<char*>(static_cast<const char*>(ws));   // twiddles only are read from ws
    return p.precision == 0 ? field_table<double>(p, b, static_cast<cplx<double>*>(out), 1, s)
                            : field_table<float>(p, b, static_cast<cplx<float>*>(out), 1, s);
}

hipError_t launch_h_scale(const Plan& p, void* ws, void* h, hipStream_t s) {
    if (p.precision != 1) return hipErrorInvalidValue;
    char* b = static_cast<char*>(ws);
    float* scale = reinterpret_cast<float*>(b + p.off_hscale);
    unsigned* emax = reinterpret_cast<unsigned*>(b + p.off_hscale + 64);
    hipLaunchKernelGGL(k_hscale_clear, dim3(1), dim3(kBlock), 0, s, emax, p.nzh);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int bs = kBlock / p.nzh * p.nzh;                     // a multiple of N_z/2
    if (bs == 0) return hipErrorInvalidValue;
    const size_t n = (size_t)p.N[0] * p.N[1] * p.nzh;
    const int grid = (int)std::min<size_t>((n + bs - 1) / bs, 256);
    hipLaunchKernelGGL(k_hscale_emax<float>, dim3(grid), dim3(bs), 0, s, p,
                       reinterpret_cast<const cplx<float>*>(b + p.off_ehat), emax);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    float* qsum = reinterpret_cast<float*>(b + p.off_hscale + 64 + (size_t)p.nzh * sizeof(unsigned));
    hipLaunchKernelGGL(k_hscale_qmax<float>, dim3(p.nzh), dim3(kBlock), 0, s, p,
                       reinterpret_cast<const cplx<float>*>(b + p.off_qhat), qsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_hscale_finish, dim3(1), dim3(kBlock), 0, s, p.nzh, emax, qsum, scale,
                       reinterpret_cast<float*>(static_cast<char*>(h) + p.h_values_bytes));
    return hipGetLastError();
}

hipError_t launch_synthesis(const Plan& p, void* ws, void* h, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    return p.precision == 0 ? synthesis<double>(p, b, h, s) : synthesis<float>(p, b, h, s);
}

}  // namespace wt
