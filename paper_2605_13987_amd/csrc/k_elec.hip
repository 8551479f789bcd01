// Readout electronics and timing features: the workflow's last step
// (Section 2) convolves the induced currents with the transfer function of
// the front end and adds noise; here, for each track, v = dt (g * i) + sigma
// noise on the time grid, then the signed amplitude, the parabola-refined
// peak time and the constant-fraction time.  The front-end impulse response g
// and the noise samples are the caller's.  One workgroup per track; the
// current row and the response are staged in LDS.
#include "common.hpp"

namespace wt {

namespace {

constexpr int kElecBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kElecBlock)
k_electronics(int nt, T dt, const T* cur, const T* g, const T* noise, T sigma, T frac, T* v_out, T* feat) {
    __shared__ T si[kMaxTime], sg[kMaxTime], sv[kMaxTime];
    __shared__ T best_a[kElecBlock];
    __shared__ int best_n[kElecBlock];
    const int k = blockIdx.x;
    const T* ik = cur + (size_t)k * nt;
    for (int n = threadIdx.x; n < nt; n += kElecBlock) {
        si[n] = ik[n];
        sg[n] = g[n];
    }
    __syncthreads();
    // v[n] = dt sum_{m<=n} g[n-m] i[m] + sigma noise[n]; first index of max |v|
    // per thread, a NaN counting as the largest value (the first NaN wins, as
    // in an argmax that propagates NaN), so that a record of NaN currents
    // still names a sample
    T ba = (T)-1;
    int bn = nt;
    for (int n = threadIdx.x; n < nt; n += kElecBlock) {
        T acc = (T)0;
        for (int m = 0; m <= n; ++m) acc += sg[n - m] * si[m];
        T v = dt * acc;
        if (noise) v += sigma * noise[(size_t)k * nt + n];
        sv[n] = v;
        v_out[(size_t)k * nt + n] = v;
        const T a = fabs(v);
        if (!isnan(ba) && (isnan(a) || a > ba)) {
            ba = a;
            bn = n;
        }
    }
    best_a[threadIdx.x] = ba;
    best_n[threadIdx.x] = bn;
    __syncthreads();
    for (int h = kElecBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            const T a1 = best_a[threadIdx.x];
            const int n1 = best_n[threadIdx.x];
            const T a2 = best_a[threadIdx.x + h];
            const int n2 = best_n[threadIdx.x + h];
            const bool nan1 = isnan(a1), nan2 = isnan(a2);
            const bool take = nan1 ? (nan2 && n2 < n1) : (nan2 || a2 > a1 || (a2 == a1 && n2 < n1));
            if (take) {
                best_a[threadIdx.x] = a2;
                best_n[threadIdx.x] = n2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // every sample n < nt was examined by some thread, so np < nt
        const int np = best_n[0] < nt ? best_n[0] : 0;
        const T amp = sv[np];
        T* f = feat + (size_t)k * 3;
        f[0] = amp;
        if (amp == (T)0) {
            f[1] = (T)np * dt;
            f[2] = (T)NAN;
            return;
        }
        const T s = amp > (T)0 ? (T)1 : (T)-1;
        T d = (T)0;
        if (np > 0 && np < nt - 1) {
            const T um = s * sv[np - 1], u0 = s * sv[np], up = s * sv[np + 1];
            const T den = um - (T)2 * u0 + up;
            if (den < (T)0) d = (um - up) / ((T)2 * den);
        }
        f[1] = ((T)np + d) * dt;
        const T thr = frac * fabs(amp);
        T t_cfd = (T)NAN;
        for (int n = np - 1; n >= 0; --n) {
            const T u = s * sv[n];
            if (u < thr) {
                t_cfd = ((T)n + (thr - u) / (s * sv[n + 1] - u)) * dt;
                break;
            }
        }
        f[2] = t_cfd;
    }
}

template <typename T>
hipError_t electronics(int n_tracks, int nt, double dt, const void* cur, const void* g, const void* noise,
                       double sigma, double frac, void* v, void* feat, hipStream_t s) {
    hipLaunchKernelGGL(k_electronics<T>, dim3(n_tracks), dim3(kElecBlock), 0, s, nt, (T)dt,
                       static_cast<const T*>(cur), static_cast<const T*>(g), static_cast<const T*>(noise),
                       (T)sigma, (T)frac, static_cast<T*>(v), static_cast<T*>(feat));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_electronics(int precision, int n_tracks, int nt, double dt, const void* cur, const void* g,
                              const void* noise, double sigma, double frac, void* v, void* feat, hipStream_t s) {
    return precision == 0 ? electronics<double>(n_tracks, nt, dt, cur, g, noise, sigma, frac, v, feat, s)
                          : electronics<float>(n_tracks, nt, dt, cur, g, noise, sigma, frac, v, feat, s);
}

}  // namespace wt
