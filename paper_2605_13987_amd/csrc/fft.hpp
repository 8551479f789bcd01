// Workgroup-cooperative inverse complex FFTs in LDS (unnormalised,
// exp(+2 pi i k n / N)), mixed radix 2/3/4/5, Stockham autosort.
//
// A length-N transform is done in passes; a pass of radix r with p = product
// of the radices already applied maps, for every i < N/r with k = i mod p,
//   x_q = a[i + q N/r] * w^(q k N/(p r)),  q < r,      w = exp(+2 pi i / N)
//   y_s = sum_q x_q exp(+2 pi i q s / r)
//   b[(i - k) r + k + s p] = y_s
// which leaves the result in natural order after the last pass.
#pragma once

#include "common.hpp"

namespace wt {

template <typename T>
struct Rad {
    static constexpr T c5_1 = (T)0.30901699437494742410;    // cos(2 pi/5)
    static constexpr T s5_1 = (T)0.95105651629515357212;    // sin(2 pi/5)
    static constexpr T c5_2 = (T)-0.80901699437494742410;   // cos(4 pi/5)
    static constexpr T s5_2 = (T)0.58778525229247312917;    // sin(4 pi/5)
    static constexpr T s3 = (T)0.86602540378443864676;      // sin(2 pi/3)
};

template <typename T, int R>
__device__ inline void butterfly(cplx<T>* x) {
    if constexpr (R == 2) {
        const cplx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = a - b;
    } else if constexpr (R == 3) {
        const cplx<T> t = x[1] + x[2], u = x[1] - x[2];
        const cplx<T> m = x[0] - scale(t, (T)0.5);
        const cplx<T> iu = mul_i(scale(u, Rad<T>::s3));
        x[0] = x[0] + t;
        x[1] = m + iu;
        x[2] = m - iu;
    } else if constexpr (R == 4) {
        const cplx<T> a = x[0] + x[2], b = x[0] - x[2], c = x[1] + x[3], d = x[1] - x[3];
        x[0] = a + c;
        x[2] = a - c;
        x[1] = b + mul_i(d);
        x[3] = b - mul_i(d);
    } else {
        const cplx<T> t1 = x[1] + x[4], t2 = x[2] + x[3], t3 = x[1] - x[4], t4 = x[2] - x[3];
        const cplx<T> a1 = x[0] + scale(t1, Rad<T>::c5_1) + scale(t2, Rad<T>::c5_2);
        const cplx<T> a2 = x[0] + scale(t1, Rad<T>::c5_2) + scale(t2, Rad<T>::c5_1);
        const cplx<T> b1 = mul_i(scale(t3, Rad<T>::s5_1) + scale(t4, Rad<T>::s5_2));
        const cplx<T> b2 = mul_i(scale(t3, Rad<T>::s5_2) - scale(t4, Rad<T>::s5_1));
        x[0] = x[0] + t1 + t2;
        x[1] = a1 + b1;
        x[4] = a1 - b1;
        x[2] = a2 + b2;
        x[3] = a2 - b2;
    }
}

template <typename T, int R>
__device__ inline void stockham_pass(const cplx<T>* a, cplx<T>* b, int N, int nfft, int p,
                                     const cplx<T>* tw, int tid, int nthr) {
    const int m = N / R;
    const int tws = N / (p * R);
    for (int idx = tid; idx < nfft * m; idx += nthr) {
        const int f = idx / m;
        const int i = idx - f * m;
        const int k = i % p;
        const cplx<T>* src = a + f * N;
        cplx<T> x[R];
#pragma unroll
        for (int q = 0; q < R; ++q) x[q] = src[i + q * m];
        if (k != 0) {
#pragma unroll
            for (int q = 1; q < R; ++q) x[q] = x[q] * tw[q * k * tws];
        }
        butterfly<T, R>(x);
        cplx<T>* dst = b + f * N + (i - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) dst[q * p] = x[q];
    }
}

// stockham_pass with the transform length N and the span P of the passes
// already applied fixed at compile time: the index arithmetic becomes shifts
// and masks (N a power of two).
template <typename T, int R, int N, int P>
__device__ inline void stockham_pass_pow2(const cplx<T>* a, cplx<T>* b, int nfft, const cplx<T>* tw, int tid,
                                          int nthr) {
    constexpr int m = N / R;
    constexpr int tws = N / (P * R);
    for (int idx = tid; idx < nfft * m; idx += nthr) {
        const int f = idx / m;
        const int i = idx - f * m;
        const int k = i % P;
        const cplx<T>* src = a + f * N;
        cplx<T> x[R];
#pragma unroll
        for (int q = 0; q < R; ++q) x[q] = src[i + q * m];
        if (k != 0) {
#pragma unroll
            for (int q = 1; q < R; ++q) x[q] = x[q] * tw[q * k * tws];
        }
        butterfly<T, R>(x);
        cplx<T>* dst = b + f * N + (i - k) * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) dst[q * P] = x[q];
    }
}

// nfft transforms of length N stored back to back in a; b is scratch of the
// same size.  Returns the buffer holding the result.  Ends with a barrier.
template <typename T>
__device__ cplx<T>* fft_inverse_lds(cplx<T>* a, cplx<T>* b, int N, int nfft, const int* rad, int nrad,
                                    const cplx<T>* tw) {
    int p = 1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int s = 0; s < nrad; ++s) {
        const int r = rad[s];
        switch (r) {
            case 4: stockham_pass<T, 4>(a, b, N, nfft, p, tw, tid, nthr); break;
            case 2: stockham_pass<T, 2>(a, b, N, nfft, p, tw, tid, nthr); break;
            case 3: stockham_pass<T, 3>(a, b, N, nfft, p, tw, tid, nthr); break;
            default: stockham_pass<T, 5>(a, b, N, nfft, p, tw, tid, nthr); break;
        }
        __syncthreads();
        cplx<T>* t = a;
        a = b;
        b = t;
        p *= r;
    }
    return a;
}

// fft_inverse_lds for a power of two N known at compile time, with the
// radices in factorize()'s order (4 while four divides what is left, then 2),
// so that the results equal the general form's bit for bit.
template <typename T, int N, int P = 1>
__device__ cplx<T>* fft_inverse_lds_pow2(cplx<T>* a, cplx<T>* b, int nfft, const cplx<T>* tw) {
    if constexpr (P >= N) {
        return a;
    } else {
        constexpr int R = (N / P) % 4 == 0 ? 4 : 2;
        stockham_pass_pow2<T, R, N, P>(a, b, nfft, tw, threadIdx.x, blockDim.x);
        __syncthreads();
        return fft_inverse_lds_pow2<T, N, P * R>(b, a, nfft, tw);
    }
}

}  // namespace wt

namespace wt {

// exp(+2 pi i j / 32) from the first octant by symmetry, so that the
// quarter-turn values are exact.
__host__ __device__ constexpr double cos_2pi_32(int j) {
    constexpr double c[9] = {1.0,
                             0.98078528040323044913,   // cos(pi/16)
                             0.92387953251128675613,   // cos(pi/8)
                             0.83146961230254523708,   // cos(3pi/16)
                             0.70710678118654752440,   // cos(pi/4)
                             0.55557023301960222474,   // cos(5pi/16)
                             0.38268343236508977173,   // cos(3pi/8)
                             0.19509032201612826785,   // cos(7pi/16)
                             0.0};
    j &= 31;
    return j <= 8 ? c[j] : (j <= 16 ? -c[16 - j] : (j <= 24 ? -c[j - 16] : c[32 - j]));
}

__host__ __device__ constexpr int bit_reverse(int i, int n) {
    int r = 0;
    for (int b = 1; b < n; b <<= 1) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

// In-register inverse DFT of R = 2, 4, 8, 16 or 32 points (radix-2, decimation
// in time, natural-order output): x[n] <- sum_k x[k] exp(+2 pi i n k / R).
template <typename T, int R>
__device__ inline void dft_reg(cplx<T>* x) {
    static_assert(R == 2 || R == 4 || R == 8 || R == 16 || R == 32, "register DFT size");
#pragma unroll
    for (int i = 0; i < R; ++i) {
        const int j = bit_reverse(i, R);
        if (j > i) {
            const cplx<T> t = x[i];
            x[i] = x[j];
            x[j] = t;
        }
    }
#pragma unroll
    for (int len = 2; len <= R; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int i = 0; i < R; i += len) {
#pragma unroll
            for (int j = 0; j < half; ++j) {
                const int m = j * (32 / len);              // exp(+2 pi i j / len) = w32^m
                const cplx<T> u = x[i + j], v = x[i + j + half];
                if (m == 0) {
                    x[i + j] = u + v;
                    x[i + j + half] = u - v;
                } else if (m == 8) {
                    x[i + j] = u + mul_i(v);
                    x[i + j + half] = u - mul_i(v);
                } else {
                    // a = u + w v with the products fused into the sums, and
                    // u - w v = 2u - a
                    const T c = (T)cos_2pi_32(m), s = (T)cos_2pi_32(m - 8);
                    const cplx<T> a{fma(v.re, c, fma(-v.im, s, u.re)), fma(v.re, s, fma(v.im, c, u.im))};
                    x[i + j] = a;
                    x[i + j + half] = cplx<T>{fma((T)2, u.re, -a.re), fma((T)2, u.im, -a.im)};
                }
            }
        }
    }
}

// cos and sin of 2 pi j / R for compile-time constants: the angle is reduced
// with integer arithmetic to q quarter turns plus x in [0, pi/4], and x goes
// through the Taylor series (14 terms: the remainder is below 1e-30), so
// that quarter turns are exact.
struct UnitRoot {
    double c, s;
};
__host__ __device__ constexpr double taylor_sin(double x) {
    double t = x, s = x;
    for (int n = 1; n < 14; ++n) {
        t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
        s += t;
    }
    return s;
}
__host__ __device__ constexpr double taylor_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int n = 1; n < 14; ++n) {
        t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
        s += t;
    }
    return s;
}
__host__ __device__ constexpr UnitRoot unit_root(int j, int R) {
    constexpr double kHalfPi = 1.57079632679489661923;
    j %= R;
    if (j < 0) j += R;
    const int q = 4 * j / R, f = 4 * j - q * R;               // angle = (pi/2) (q + f/R)
    double c = 0.0, s = 0.0;
    if (2 * f <= R) {
        const double x = kHalfPi * f / R;
        c = taylor_cos(x);
        s = taylor_sin(x);
    } else {
        const double x = kHalfPi * (R - f) / R;                // (pi/2) f/R = pi/2 - x
        c = taylor_sin(x);
        s = taylor_cos(x);
    }
    if (q == 0) return UnitRoot{c, s};
    if (q == 1) return UnitRoot{-s, c};
    if (q == 2) return UnitRoot{-c, -s};
    return UnitRoot{s, -c};
}

// x exp(+2 pi i e / R) for compile-time e and R (quarter turns as swaps).
template <typename T>
__device__ inline cplx<T> mul_unit_root(const cplx<T>& x, int e, int R) {
    e %= R;
    if (e == 0) return x;
    if (2 * e == R) return cplx<T>{-x.re, -x.im};
    if (4 * e == R) return mul_i(x);
    if (4 * e == 3 * R) return cplx<T>{x.im, -x.re};
    const UnitRoot w = unit_root(e, R);
    const T c = (T)w.c, s = (T)w.s;
    return cplx<T>{fma(x.re, c, -x.im * s), fma(x.re, s, x.im * c)};
}

template <int L>
__host__ __device__ constexpr int first_radix() {
    return L % 4 == 0 ? 4 : (L % 2 == 0 ? 2 : (L % 3 == 0 ? 3 : 5));
}

// In-register inverse DFT of a 2,3,5-smooth R (the Stockham passes of
// fft_inverse_lds with compile-time indices: radix 4 first, then 2, 3, 5; the
// copies between passes are register renames).  P: product of the radices
// already applied.
template <typename T, int R, int P>
__device__ inline void dft_mixed_pass(cplx<T>* a) {
    if constexpr (P < R) {
        constexpr int r = first_radix<R / P>();
        constexpr int m = R / r;
        constexpr int tws = R / (P * r);
        static_assert(R % (P * r) == 0 && (r == 2 || r == 3 || r == 4 || r == 5), "smooth register DFT");
        cplx<T> b[R];
#pragma unroll
        for (int i = 0; i < m; ++i) {
            const int k = i % P;
            cplx<T> x[r];
#pragma unroll
            for (int q = 0; q < r; ++q) x[q] = mul_unit_root(a[i + q * m], q * k * tws, R);
            butterfly<T, r>(x);
#pragma unroll
            for (int s = 0; s < r; ++s) b[(i - k) * r + k + s * P] = x[s];
        }
#pragma unroll
        for (int i = 0; i < R; ++i) a[i] = b[i];
        dft_mixed_pass<T, R, P * r>(a);
    }
}

// x[n] <- sum_k x[k] exp(+2 pi i n k / R) in registers, any R the synthesis uses.
template <typename T, int R>
__device__ inline void dft_any(cplx<T>* x) {
    if constexpr ((R & (R - 1)) == 0)
        dft_reg<T, R>(x);
    else
        dft_mixed_pass<T, R, 1>(x);
}

}  // namespace wt
