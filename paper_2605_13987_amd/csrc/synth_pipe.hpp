// Register-FFT synthesis of H along z (the per-column step of the bulk
// field: H_a(X, Y, z, t) = sum_{m_z} exp(i k_z z) sum_w Ehat_a(X - X_w, Y - Y_w,
// m_z) Qhat_w(m_z, t), a Hermitian inverse FFT of length N_z per (X, Y, t, a);
// Section 3's spectral extension to the bulk).  Included by the sources that
// instantiate it: k_bulk.hip (powers of two) and k_synth_smooth.hip (other
// 2,3,5-smooth sizes).
#pragma once

#include "fft.hpp"

#include <type_traits>

namespace wt {

namespace {
// p advanced by a 32-bit byte offset: with p uniform over the wavefront this
// is the scalar-base + lane-offset form of global memory access.
template <typename T>
__device__ inline T* byte_offset(T* p, unsigned off) {
    return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + off);
}
template <typename T>
__device__ inline const T* byte_offset(const T* p, unsigned off) {
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + off);
}

typedef float vec4f __attribute__((ext_vector_type(4)));
typedef float vec2f __attribute__((ext_vector_type(2)));
typedef _Float16 vec2h __attribute__((ext_vector_type(2)));
typedef double vec2d __attribute__((ext_vector_type(2)));

constexpr int const_gcd(int a, int b) { return b == 0 ? a : const_gcd(b, a % b); }

// Synthesis of H(X, Y, z, t) for N_z = N1 x N2, with the length-N_z
// transforms done in registers.  One workgroup per (X, Y) column; H is
// produced in blocks of TB samples (16, or 8), each staged whole in LDS as
// [z][sample][component] (the row layout is described at PipeShape):
//
// 1. Spectra.  A memory-team thread owns k_z index kk and keeps the field
//    table entries Ehat_a(X - X_w, Y - Y_w, kk) of all components and columns
//    in registers.  For a pair of samples (t, t+1) it writes the spectrum of
//    the complex signal that carries both, Z(kk) = F_t(kk) + i F_{t+1}(kk)
//    with F_t(kk) = sum_w Ehat_w Qhat_w(kk, t), to row kk, and
//    Z(N_z - kk) = conj F_t(kk) + i conj F_{t+1}(kk) to row N_z - kk.
// 2. Transforms.  A group of N1 lanes of the transform team (inside one
//    wavefront) owns one complex FFT of length N_z.  Pass 1: lane k1 reads
//    Z[k1 + N1 k2] (k2 < N2; Z(N_z/2) = 0), transforms over k2, applies
//    exp(+2 pi i n2 k1 / N_z) (twiddles kept in registers) and writes
//    element (k1, n2) to row k1 N2 + n2.  Pass 2: lane j transforms over k1
//    for the columns n2 = j + N1 c < N2 and writes sample z = n2 + N2 n1.  The
//    real and imaginary parts are samples t and t+1 of H_a(z).  All lanes of
//    a group read before any writes back, in program order of their
//    wavefront.  Every LDS address is a per-lane base plus a constant.
// 3. Copy-out.  The finished block is one contiguous run of H, written by
//    the memory team with non-temporal stores (H is not re-read here and
//    should not evict the tables from L2).
//
// Two staging buffers and two teams of wavefronts overlap the steps: while
// the transform team runs pass 1 and then pass 2 of block s in buffer
// s mod 2, the memory team loads the column spectra of block s+1 and copies
// block s-1 out of the other buffer (phase 1), then builds block s+1's
// spectra into it (phase 2).  A workgroup barrier ends each phase; within a
// phase the teams touch different buffers.
template <typename T, int N1, int N2, int WC, typename TO, int TB>
__global__ void __launch_bounds__(pipe_shape_for(N1 * N2, N1, TB).threads)
k_synthesis_pipe(Plan p, const cplx<T>* ehat, const cplx<T>* qhat, const cplx<T>* twz, const float* h_scale,
                 TO* H) {
    // Issue priority above the current's binning, which can run beside this
    // launch on another stream: 256 x 256 x 512 step 65.2 -> 64.5 ms (the
    // synthesis 40.3 -> 39.6 ms; the binning still ends within it).
    __builtin_amdgcn_s_setprio(3);
    constexpr int NZ = N1 * N2;
    constexpr int NZH = NZ / 2;
    constexpr PipeShape SH = pipe_shape_for(NZ, N1, TB);
    constexpr int C = (N2 + N1 - 1) / N1;                      // pass-2 columns per lane
    constexpr int CP = N2 % N1 == 0 ? N2 / N1 : 1;             // rows k1 + N1 k2: (k2 / CP) N2-runs
    constexpr int TBC = SH.tbc;                                // samples per block
    constexpr int NP = TBC / 2;                                // sample pairs per block
    constexpr int NG = 3 * NP;                                 // transforms per block
    constexpr int GPW = SH.gpw;                                // transform groups per wavefront
    constexpr int NTT = SH.ntt;                                // transform team
    constexpr int NTM = SH.ntm;                                // memory team
    constexpr int NTA = SH.ntm_act;                            // its threads that own a k_z
    constexpr int GAP = SH.gap;
    constexpr int RS = SH.rs;
    constexpr int PAD = SH.pad;                                // row z at z RS + (z / N2) PAD
    constexpr int BUF = SH.buffer;                             // elements per staging buffer
    constexpr int PPT = SH.ppt;                                // pairs covered by one pass of the team
    constexpr int PFI = (NP + PPT - 1) / PPT;                  // (kk, pair) items per thread
    constexpr int LW = 3 * TBC / 2;                            // value pairs per row
    // Copy-out: value pair p = lane + NTM k of the block (row p / LW); with
    // CR = LW / gcd(NTM, LW) per-lane bases, store k = CR j + r sits CROWS j
    // rows after base r, a constant offset.
    constexpr int CR = LW / const_gcd(NTM, LW);
    constexpr int CROWS = NTM * CR / LW;
    constexpr int CJ = (NZ + CROWS - 1) / CROWS;
    // Z(N_z/2) = Z[K1H + N1 K2H]
    constexpr int K1H = NZH % N1, K2H = NZH / N1;
    static_assert(SH.n1 == N1 && SH.n2 == N2 && NTT % 64 == 0 && NTM % 64 == 0 && GPW * N1 <= 64 &&
                      pipe_fits(SH, (int)sizeof(T)),
                  "synthesis split");
    static_assert(NTA % NZH == 0 && NTA <= NTM && NTT >= (NG + GPW - 1) / GPW * 64, "synthesis teams");
    static_assert(PAD == 0 || (N2 % N1 == 0 && NZ % CROWS == 0 && (N2 % CROWS == 0 || CROWS % N2 == 0)),
                  "synthesis row padding");
    static_assert(GAP % 2 == 0, "synthesis thread mapping");
    extern __shared__ __align__(16) unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    const int Nx = p.N[0], Ny = p.N[1], nt = p.n_time;
    const int col = blockIdx.x;
    const int ix = col / Ny, iy = col - (col / Ny) * Ny;
    TO* hcol = H + (size_t)col * NZ * nt * 3;
    const int nblk = (nt + TBC - 1) / TBC;
    // stored value = H * enc (float16 H), else H
    constexpr bool kScaled = !std::is_same<TO, T>::value;
    // column of sample pair q (component 0, real part): 6 q, plus the gap in the second half
    auto pcol = [](int q) { return 6 * q + (q >= NP / 2 ? GAP : 0); };
    auto settle = [](const cplx<T>& v) { asm volatile("" ::"v"(v.re), "v"(v.im)); };

    if (threadIdx.x < NTT) {
        // ------------------------------------------------ transform team
        const int lane = threadIdx.x & 63;
        const int g = (threadIdx.x >> 6) * GPW + lane / N1;
        const int k1 = lane % N1;
        // lanes past the wavefront's last whole group, and groups past the
        // block's transforms, only take part in the barriers
        const bool tact = lane < GPW * N1 && g < NG;
        const int hg = g >> 1, sg = g & 1;
        const int a = hg % 3, tp = hg / 3 + sg * (NP / 2);
        cplx<T> twr[N2];                                       // exp(+2 pi i n2 k1 / N_z)
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) twr[n2] = twz[n2 * k1];
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) settle(twr[n2]);
        // pass 1: Z[k1 + N1 k2] is row k1 + N1 k2, at k1 RS + N1 k2 RS + (k2 / CP) PAD;
        // element (k1, n2) goes to row k1 N2 + n2, at k1 (N2 RS + PAD) + n2 RS
        auto pass1 = [&](T* stage, int npair) {
            if (!tact || tp >= npair) return;
            // lane indices re-derived per block (opaque to the optimiser) so that
            // the per-lane LDS addresses are not hoisted out of the block loop
            int kl = (threadIdx.x & 63) % N1, slot = pcol(tp) + a;
            asm volatile("" : "+v"(kl), "+v"(slot));
            const T* rd = stage + slot + kl * RS;
            cplx<T> x[N2];
#pragma unroll
            for (int k2 = 0; k2 < N2; ++k2) {
                const int o = N1 * k2 * RS + (k2 / CP) * PAD;
                x[k2] = cplx<T>{rd[o], rd[o + 3]};
            }
            if (kl == K1H) x[K2H] = cplx<T>{(T)0, (T)0};        // Z(N_z/2) = 0
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            dft_any<T, N2>(x);
            T* wr = stage + slot + kl * (N2 * RS + PAD);
#pragma unroll
            for (int n2 = 0; n2 < N2; ++n2) {
                cplx<T> y = x[n2];
                if (n2 != 0) y = y * twr[n2];
                wr[n2 * RS] = y.re;
                wr[n2 * RS + 3] = y.im;
            }
        };
        // pass 2: lane j takes the columns n2 = j + N1 c < N2; element (k1', n2) is at
        // k1' (N2 RS + PAD) + N1 c RS + j RS, and sample z = n2 + N2 n1 goes to
        // row z, at j RS + (N1 c + N2 n1) RS + n1 PAD
        auto pass2 = [&](T* stage, int npair) {
            if (!tact || tp >= npair) return;
            int kl = (threadIdx.x & 63) % N1, slot = pcol(tp) + a;
            asm volatile("" : "+v"(kl), "+v"(slot));
            T* rw = stage + slot + kl * RS;
            // column c of this lane exists (always, when N1 divides N2)
            auto has = [&](int c) { return C * N1 == N2 || kl + N1 * c < N2; };
            cplx<T> v[C][N1];
#pragma unroll
            for (int c = 0; c < C; ++c)
#pragma unroll
                for (int j = 0; j < N1; ++j) {
                    const int o = j * (N2 * RS + PAD) + N1 * c * RS;
                    v[c][j] = has(c) ? cplx<T>{rw[o], rw[o + 3]} : cplx<T>{(T)0, (T)0};
                }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (!has(c)) continue;
                dft_any<T, N1>(v[c]);
#pragma unroll
                for (int n1 = 0; n1 < N1; ++n1) {
                    const int o = (N1 * c + N2 * n1) * RS + n1 * PAD;
                    rw[o] = v[c][n1].re;
                    rw[o + 3] = v[c][n1].im;
                }
            }
        };
        __syncthreads();                                       // block 0 staged
        for (int s = 0; s < nblk; ++s) {
            const int npair = (min(TBC, nt - s * TBC) + 1) / 2;
            T* stage = lds + (s & 1) * BUF;
            pass1(stage, npair);
            __syncthreads();
            pass2(stage, npair);
            __syncthreads();
        }
    } else {
        // --------------------------------------------------- memory team
        const int m = threadIdx.x - NTT;
        const T enc = kScaled ? (T)h_scale[0] : (T)1;
        const int kkb = m % NZH;
        const bool mact = NTA == NTM || m < NTA;               // owns k_z kkb and pairs pb + PPT k
        int pb = m / NZH;                                      // first sample pair of this thread
        if constexpr (NZH % 64 == 0) pb = __builtin_amdgcn_readfirstlane(pb);
        cplx<T> e[3][WC];
#pragma unroll
        for (int w = 0; w < WC; ++w) {
            const int sx = (ix - p.col[w].ix + Nx) % Nx;
            const int sy = (iy - p.col[w].iy + Ny) % Ny;
            const cplx<T>* src = ehat + (((size_t)sx * Ny + sy) * NZH + kkb) * 3;
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) e[aa][w] = src[aa];
        }
#pragma unroll
        for (int w = 0; w < WC; ++w)
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) settle(e[aa][w]);
        cplx<T> pq[PFI][WC][2];
        auto settle_all = [&]() {
#pragma unroll
            for (int k = 0; k < PFI; ++k)
#pragma unroll
                for (int w = 0; w < WC; ++w) {
                    settle(pq[k][w][0]);
                    settle(pq[k][w][1]);
                }
        };
        // Column spectra Qhat_w(kkb, t) of both samples of this thread's pairs
        // of the block at t0.  A sample past the block is zero when it pairs
        // with the last one (odd block length); pairs wholly past the block
        // are not used.
        auto fetch = [&](int t0) {
            if (!mact) return;
            const int tbl = min(TBC, nt - t0);
#pragma unroll
            for (int k = 0; k < PFI; ++k)
#pragma unroll
                for (int sm = 0; sm < 2; ++sm) {
                    const int tin = 2 * (pb + k * PPT) + sm;
                    if (tin < tbl) {
                        const cplx<T>* q = qhat + (size_t)(t0 + tin) * WC * NZH;
#pragma unroll
                        for (int w = 0; w < WC; ++w)
                            pq[k][w][sm] = *byte_offset(q + w * NZH, kkb * sizeof(cplx<T>));
                    } else if (tin == tbl) {
#pragma unroll
                        for (int w = 0; w < WC; ++w) pq[k][w][sm] = cplx<T>{(T)0, (T)0};
                    }
                }
        };
        // spectra Z of the npair sample pairs of a block: rows kkb and
        // N_z - kkb (row N_z/2 for kk = 0, which pass 1 does not read)
        auto build = [&](T* stage, int npair) {
            settle_all();
            if (!mact) return;
            const int zm = kkb == 0 ? NZH : NZ - kkb;
            T* r0 = stage + kkb * RS + (kkb / N2) * PAD;
            T* r1 = stage + zm * RS + (zm / N2) * PAD;
#pragma unroll
            for (int k = 0; k < PFI; ++k) {
                if (pb + k * PPT < npair) {
                    // Z(kk) = sum_w Ehat_w (Qhat_w(t) + i Qhat_w(t+1)),
                    // Z(N_z - kk) = sum_w conj(Ehat_w) (conj Qhat_w(t) + i conj Qhat_w(t+1))
                    cplx<T> u[WC], v[WC];
#pragma unroll
                    for (int w = 0; w < WC; ++w) {
                        const cplx<T> q0 = pq[k][w][0], q1 = pq[k][w][1];
                        u[w] = cplx<T>{q0.re - q1.im, q0.im + q1.re};
                        v[w] = cplx<T>{q0.re + q1.im, q1.re - q0.im};
                    }
#pragma unroll
                    for (int aa = 0; aa < 3; ++aa) {
                        cplx<T> z = e[aa][0] * u[0], zr = conj(e[aa][0]) * v[0];
#pragma unroll
                        for (int w = 1; w < WC; ++w) {
                            z = z + e[aa][w] * u[w];
                            zr = zr + conj(e[aa][w]) * v[w];
                        }
                        const int c = pcol(pb + k * PPT) + aa;
                        r0[c] = z.re;
                        r0[c + 3] = z.im;
                        r1[c] = zr.re;
                        r1[c + 3] = zr.im;
                    }
                }
            }
        };
        // A full block: each lane writes two consecutive values of a row per
        // store (rows are 3 x block values, the gap falls between value
        // pairs); a fixed number of stores per thread (the last ones guarded
        // when NTM does not divide the block's value pairs), so that the
        // spectra loads issued just before are waited for without waiting for
        // the stores.
        auto copyout_full = [&](const T* stage, int t0) {
            TO* dst = hcol + (size_t)t0 * NZ * 3;
            int lane = m;
            asm volatile("" : "+v"(lane));
            const T* src[CR];
#pragma unroll
            for (int r = 0; r < CR; ++r) {
                const int pr = lane + NTM * r;
                const int z = pr / LW, rr = 2 * (pr - z * LW);
                src[r] = stage + z * RS + (z / N2) * PAD + rr + (rr >= 3 * TBC / 2 ? GAP : 0);
            }
#pragma unroll
            for (int k = 0; k < CR * CJ; ++k) {
                const int j = k / CR, r = k - j * CR;
                if ((k + 1) * NTM > NZ * LW && k * NTM + lane >= NZ * LW) continue;
                const T* sk = src[r] + j * CROWS * RS + (j * CROWS / N2) * PAD;
                TO* dk = byte_offset(dst + k * NTM * 2, lane * 2 * (unsigned)sizeof(TO));
                if constexpr (kScaled) {
                    __builtin_nontemporal_store(vec2h{(_Float16)(sk[0] * enc), (_Float16)(sk[1] * enc)},
                                                reinterpret_cast<vec2h*>(dk));
                } else if constexpr (sizeof(T) == 4) {
                    __builtin_nontemporal_store(vec2f{sk[0], sk[1]}, reinterpret_cast<vec2f*>(dk));
                } else {
                    __builtin_nontemporal_store(vec2d{sk[0], sk[1]}, reinterpret_cast<vec2d*>(dk));
                }
            }
            settle_all();
        };
        auto copyout = [&](const T* stage, int t0) {
            const int tbl = min(TBC, nt - t0);
            TO* dst = hcol + (size_t)t0 * NZ * 3;
            if (tbl == TBC) {
                copyout_full(stage, t0);
            } else {
                const int rowlen = tbl * 3;
                const int dz = NTM / rowlen, dr = NTM - dz * rowlen;
                int z = m / rowlen, r = m - (m / rowlen) * rowlen;
                for (int idx = m; idx < NZ * rowlen; idx += NTM) {
                    const T v = stage[z * RS + (z / N2) * PAD + r + (r >= 3 * TBC / 2 ? GAP : 0)];
                    __builtin_nontemporal_store(kScaled ? (TO)(v * enc) : (TO)v, dst + idx);
                    z += dz;
                    r += dr;
                    if (r >= rowlen) {
                        r -= rowlen;
                        ++z;
                    }
                }
            }
        };
        // Block s (>= 1) of the loop copies out block s-1, which is full (only
        // the last block can be partial), after issuing the loads of block
        // s+1: every spectra load is followed by the same number of stores
        // and waited for right after them, and nothing left pending crosses
        // a loop iteration.
        fetch(0);
        build(lds, (min(TBC, nt) + 1) / 2);
        __syncthreads();                                       // block 0 staged
        if (TBC < nt) fetch(TBC);
        __syncthreads();                                       // pass 1 of block 0 done
        if (TBC < nt) build(lds + BUF, (min(TBC, nt - TBC) + 1) / 2);
        settle_all();
        __syncthreads();                                       // block 0 transformed
        for (int s = 1; s < nblk; ++s) {
            const int tn = (s + 1) * TBC;
            if (tn < nt) fetch(tn);
            copyout_full(lds + ((s - 1) & 1) * BUF, (s - 1) * TBC);
            __syncthreads();                                   // pass 1 of block s done
            if (tn < nt) build(lds + ((s + 1) & 1) * BUF, (min(TBC, nt - tn) + 1) / 2);
            __syncthreads();                                   // block s transformed
        }
        copyout(lds + ((nblk - 1) & 1) * BUF, (nblk - 1) * TBC);
    }
}

template <typename T, int N1, int N2, int WC, typename TO, int TB>
hipError_t synthesis_pipe(const Plan& p, char* b, void* h, hipStream_t s) {
    constexpr PipeShape SH = pipe_shape_for(N1 * N2, N1, TB);
    const size_t lds = pipe_lds(SH, sizeof(T));
    hipError_t err = hipFuncSetAttribute((const void*)k_synthesis_pipe<T, N1, N2, WC, TO, TB>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL((k_synthesis_pipe<T, N1, N2, WC, TO, TB>), dim3(p.N[0] * p.N[1]), dim3(SH.threads), lds, s, p,
                       reinterpret_cast<const cplx<T>*>(b + p.off_ehat),
                       reinterpret_cast<const cplx<T>*>(b + p.off_qhat),
                       reinterpret_cast<const cplx<T>*>(b + p.off_tw[2]),
                       reinterpret_cast<const float*>(b + p.off_hscale), static_cast<TO*>(h));
    return hipGetLastError();
}

}  // namespace

}  // namespace wt
