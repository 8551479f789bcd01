// Adjoint of the path: the gradient of a loss L(i) of the Eq. 1 currents with
// respect to each column's quarter-column resistivities and radius (the
// electrode parameters of the paper's Section 5 results), given dL/di.
//
// Everything after the boundary fit is linear in the charges, so the chain
// is run backwards without forming H or its derivative:
//
// 1. Event projection.  A moving step e = (carrier c, step m) reads H at the
//    8 trilinear corners v of its midpoint, and the synthesis writes
//      H_a(v, t) = sum_w sum_{k < N_z/2} m_k Re[e^{2 pi i k z_v / N_z}
//                  Ehat_a(x_v - X_w, y_v - Y_w, k) Qhat_w(k, t)]
//    (m_0 = 1, m_k = 2).  So the current is linear in the column spectra with
//      phi_{e,w}(k) = -q_c m_k sum_v w_v e^{2 pi i k z_v / N_z} sum_a dx_a Ehat_a,
//    summed per track and step into Phi_{tr,w}(k, m).
// 2. Lag correlation: Gamma_w(k, t) = sum_tr sum_m Phi_{tr,w}(k, m) dL/di_tr(m + t),
//    so that dL/d(Re Qhat) - i dL/d(Im Qhat) = Gamma.
// 3. Adjoint z-transform: dL/dq_j(t) = sum_k Re[Gamma_w(k, t) e^{-i k_z z_j}].
// 4. Adjoint time quadrature: mu_j(f) = df c_f sum_n dL/dq_j(t_n) e^{+i w_f t_n},
//    so that dL = Re sum_f mu(f)^T dq(w_f).
// 5. Transposed boundary-fit solves S(w)^T lambda = [mu; 0] (k_solve.hip);
//    then dL/dtheta = -sum_f Re[lambda^T (dS/dtheta) [q; c]].
// 6. dS/dtheta: the RC-line block i w R_w(min(m, m')) through sigma_w and r_w,
//    reduced per frequency with suffix sums (sum_{i,j} l_i min(m_i, m_j) q_j =
//    sum_{l >= 1} (sum_{m >= l} l_m)(sum_{m >= l} q_m)), and the collocation
//    matrix through r (collocation offset of its rows, source width r/4 of its
//    columns), contracted with K_ij = sum_f Re[lambda_i q_j].
// 7. Pitch: a uniform scaling by s of the in-plane cell size, the column axes
//    and the carriers' in-plane coordinates.  The trilinear weights and the
//    column spectra are unchanged; the current changes at fixed charges
//    through the field table (dEhat/ds) and the in-plane displacements, i.e.
//    by the projections phi^s = -q m_k sum_v w_v e^{...} (dx . dEhat/ds +
//    dx_x Ehat_x + dx_y Ehat_y), which give dL/ds = sum_{t,w,k} Re[Gamma^s
//    Qhat]; and the boundary fit through dA/ds (a third lattice-sum table and
//    -2 A from the cell volume), taken with lambda as in step 6.
#include "common.hpp"

#include <algorithm>

namespace wt {

namespace {

constexpr int kBlock = 256;

using c64 = cplx<double>;

__device__ inline c64 cinv(c64 a) {
    const double d = a.re * a.re + a.im * a.im;
    return d == 0.0 ? c64{0.0, 0.0} : c64{a.re / d, -a.im / d};
}

__device__ inline double block_sum_all(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;   // valid in every thread
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_fill(T* out, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = (T)0;
}

template <typename T>
__device__ inline int wrap_cell(T f, int n) {
    const T r = f - (T)n * floor(f / (T)n);
    const int i = (int)r;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Step 1.  Block (m, carrier chunk, item group): the moving steps m of the
// chunk's carriers, one (column w, k_z) item per thread.  Sums stay in
// registers while consecutive carriers share a track and are added to Phi
// when it changes.  Consecutive carriers at one step mostly share their (x, y)
// cell (a track's carriers drift side by side), so each thread keeps the
// field table and its pitch derivative at the cell's four (x, y) corners in
// registers and reloads them only when the cell changes.  The corners and
// weights follow the forward convolution exactly.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_events(Plan p, const cplx<T>* ehat, const cplx<T>* eds, const cplx<T>* twz, int n_carriers, int n_tracks,
             const T* pos, const T* charge, const int* track, int chunk, cplx<T>* phi, cplx<T>* phis) {
    const int m = blockIdx.x;
    const int c0 = blockIdx.y * chunk;
    const int c1 = min(n_carriers, c0 + chunk);
    const int Nx = p.N[0], Ny = p.N[1], Nz = p.N[2], nzh = p.nzh, W = p.n_cols, nt = p.n_time;
    const int n_items = W * nzh;
    const int it = blockIdx.z * kBlock + threadIdx.x;
    const bool ok = it < n_items;
    const int wi = ok ? it / nzh : 0;
    const int k = ok ? it - wi * nzh : 0;
    const Column& col = p.col[wi];
    cplx<T> acc{(T)0, (T)0}, accs{(T)0, (T)0};
    cplx<T> ce[4][3], cd[4][3];                              // at (x0,y0), (x0,y1), (x1,y0), (x1,y1)
    int cx = -1, cy = -1;
    int cur = -1;
    // the step m of up to kBlock carriers at a time, loaded by all threads
    // at once (a serial loop of dependent loads would wait on each carrier)
    __shared__ T sp[kBlock][6];
    __shared__ T sq[kBlock];
    __shared__ int st[kBlock];
    auto flush = [&]() {
        const size_t o = (((size_t)cur * nt + m) * W + wi) * nzh + k;
        if (cur >= 0 && ok && (acc.re != (T)0 || acc.im != (T)0)) {
            atomicAdd(&phi[o].re, acc.re);
            atomicAdd(&phi[o].im, acc.im);
        }
        if (cur >= 0 && ok && (accs.re != (T)0 || accs.im != (T)0)) {
            atomicAdd(&phis[o].re, accs.re);
            atomicAdd(&phis[o].im, accs.im);
        }
        acc = accs = cplx<T>{(T)0, (T)0};
    };
    for (int cb = c0; cb < c1; cb += kBlock) {
        const int nb = min(kBlock, c1 - cb);
        __syncthreads();
        if ((int)threadIdx.x < nb) {
            const int c = cb + threadIdx.x;
            const T* P = pos + ((size_t)c * (nt + 1) + m) * 3;
#pragma unroll
            for (int e = 0; e < 6; ++e) sp[threadIdx.x][e] = P[e];
            sq[threadIdx.x] = charge[c];
            st[threadIdx.x] = track[c];
        }
        __syncthreads();
        for (int ci = 0; ci < nb; ++ci) {
            const int tr = st[ci];
            if (tr < 0 || tr >= n_tracks) continue;
            const T* P = sp[ci];
            const T dx = P[3] - P[0], dy = P[4] - P[1], dz = P[5] - P[2];
            if (dx == (T)0 && dy == (T)0 && dz == (T)0) continue;
            const T ux = (P[0] + P[3]) * (T)0.5 * (T)(Nx / p.L[0]);
            const T uy = (P[1] + P[4]) * (T)0.5 * (T)(Ny / p.L[1]);
            const T uz = (P[2] + P[5]) * (T)0.5 * (T)(Nz / p.L[2]);
            if (!(isfinite(ux) && isfinite(uy) && isfinite(uz))) continue;
            if (tr != cur) {
                flush();
                cur = tr;
            }
            const T flx = floor(ux), fly = floor(uy), flz = floor(uz);
            const T fx = ux - flx, fy = uy - fly, fz = uz - flz;
            const T gx = (T)1 - fx, gy = (T)1 - fy, gz = (T)1 - fz;
            const int x0 = wrap_cell(flx, Nx), y0 = wrap_cell(fly, Ny), z0 = wrap_cell(flz, Nz);
            const int z1 = z0 + 1 == Nz ? 0 : z0 + 1;
            const T q = sq[ci];
            if (!ok) continue;
            if (x0 != cx || y0 != cy) {                          // the same decision in every thread
                const int x1 = x0 + 1 == Nx ? 0 : x0 + 1;
                const int y1 = y0 + 1 == Ny ? 0 : y0 + 1;
                const int sx[2] = {(x0 - col.ix + Nx) % Nx, (x1 - col.ix + Nx) % Nx};
                const int sy[2] = {(y0 - col.iy + Ny) % Ny, (y1 - col.iy + Ny) % Ny};
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    const size_t o = (((size_t)sx[cc >> 1] * Ny + sy[cc & 1]) * nzh + k) * 3;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        ce[cc][a] = ehat[o + a];
                        cd[cc][a] = eds[o + a];
                    }
                }
                cx = x0;
                cy = y0;
            }
            // dx . Ehat at each (x, y) corner, and dx . dEhat/ds + the in-plane
            // part of dx . Ehat, weighted by the corner's in-plane weight
            const T wxy[4] = {gx * gy, gx * fy, fx * gy, fx * fy};
            cplx<T> v{(T)0, (T)0}, vs{(T)0, (T)0};
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
                const cplx<T> a = ce[cc][0], b = ce[cc][1], cz = ce[cc][2];
                const cplx<T> da = cd[cc][0], db = cd[cc][1], dc = cd[cc][2];
                const cplx<T> pxy{a.re * dx + b.re * dy, a.im * dx + b.im * dy};
                const cplx<T> pe{pxy.re + cz.re * dz, pxy.im + cz.im * dz};
                const cplx<T> ps{pxy.re + da.re * dx + db.re * dy + dc.re * dz,
                                 pxy.im + da.im * dx + db.im * dy + dc.im * dz};
                v = v + scale(pe, wxy[cc]);
                vs = vs + scale(ps, wxy[cc]);
            }
            const cplx<T> ph = scale(twz[(k * z0) % Nz], gz) + scale(twz[(k * z1) % Nz], fz);
            const T mq = k == 0 ? -q : (T)(-2) * q;
            acc = acc + scale(v * ph, mq);
            accs = accs + scale(vs * ph, mq);
        }
    }
    flush();
}

// Step 2.  One thread per (column, k_z) item and lag t.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_adj_gamma(Plan p, int n_tracks, const cplx<T>* phi, const T* grad_i, c64* gamma) {
    const int it = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    const int n_items = p.n_cols * p.nzh, nt = p.n_time;
    if (it >= n_items) return;
    double re = 0.0, im = 0.0;
    for (int tr = 0; tr < n_tracks; ++tr) {
        const T* g = grad_i + (size_t)tr * nt;
        const cplx<T>* ph = phi + (size_t)tr * nt * n_items + it;
        for (int m = 0; m + t < nt; ++m) {
            const double gv = (double)g[m + t];
            const cplx<T> v = ph[(size_t)m * n_items];
            re += gv * (double)v.re;
            im += gv * (double)v.im;
        }
    }
    gamma[(size_t)t * n_items + it] = c64{re, im};
}

__device__ inline double node_z(const Column& c, int m) {
    return c.z_contact + (m * (c.z_free - c.z_contact)) / (c.n - 1);
}

__device__ inline int column_of(const Plan& p, int i) {
    int w = 0;
    while (w + 1 < p.n_cols && i >= p.col[w + 1].offset) ++w;
    return w;
}

// Step 3.  One thread per source and time sample.
__global__ void __launch_bounds__(kBlock) k_adj_sources(Plan p, const c64* gamma, double* gbar) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int t = blockIdx.y;
    if (i >= p.n_q) return;
    const int w = column_of(p, i);
    const Column& c = p.col[w];
    const double z = node_z(c, i - c.offset);
    const c64* g = gamma + ((size_t)t * p.n_cols + w) * p.nzh;
    double acc = 0.0;
    for (int k = 0; k < p.nzh; ++k) {
        double x = k * (z / p.L[2]);
        x -= floor(x);
        double s, cs;
        sincospi(2.0 * x, &s, &cs);
        acc += g[k].re * cs + g[k].im * s;      // Re[g e^{-i k_z z}]
    }
    gbar[(size_t)t * p.n_q + i] = acc;
}

// Step 7, fixed charges: pitch[t] = sum_{w,k} Re[Gamma^s_w(k, t) Qhat_w(k, t)],
// one block per lag t.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_adj_pitch_lag(Plan p, const c64* gammas, const cplx<T>* qhat,
                                                          double* pitch) {
    __shared__ double red[kBlock / 64];
    const int t = blockIdx.x, n_items = p.n_cols * p.nzh;
    double acc = 0.0;
    for (int it = threadIdx.x; it < n_items; it += blockDim.x) {
        const c64 g = gammas[(size_t)t * n_items + it];
        const cplx<T> q = qhat[(size_t)t * n_items + it];
        acc += g.re * (double)q.re - g.im * (double)q.im;
    }
    acc = block_sum_all(acc, red);
    if (threadIdx.x == 0) pitch[t] = acc;
}

// Step 4.  One thread per unknown (the gauge row gets 0) and frequency.
__global__ void __launch_bounds__(kBlock) k_adj_rhs(Plan p, const double* gbar, c64* rhs) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (i >= p.n) return;
    c64 acc{0.0, 0.0};
    if (i < p.n_q) {
        const double r = p.df * p.dt;
        for (int n = 0; n < p.n_time; ++n) {
            double x = (double)((long long)f * n) * r;
            x -= floor(x);
            double s, c;
            sincospi(2.0 * x, &s, &c);
            const double g = gbar[(size_t)n * p.n_q + i];
            acc.re += g * c;
            acc.im += g * s;
        }
        const double cf = (f == 0 || (f == p.n_freq - 1 && p.last_weight_one)) ? 1.0 : 2.0;
        acc = scale(acc, cf * p.df);
    }
    rhs[(size_t)f * p.n + i] = acc;
}

// Step 6, RC-line terms: one block per frequency, one thread per column.
// With z_w = i w D_w / (pi r_w^2 (sigma_w + i w eps)) and T_w the suffix-sum
// contraction of lambda and q over the column's nodes,
//   dL/dsigma_w += Re[T_w z_w / (sigma_w + i w eps)],  dL/dr_w += 2 Re[T_w z_w] / r_w.
__global__ void __launch_bounds__(64) k_adj_freq(Plan p, const c64* qw, const c64* lam, double* part) {
    const int f = blockIdx.x;
    const int w = threadIdx.x;
    if (w >= p.n_cols) return;
    const Column& c = p.col[w];
    const double omega = 2.0 * kPi * p.df * f;
    const c64* lq = lam + (size_t)f * p.n + c.offset;
    const c64* qq = qw + (size_t)f * p.n + c.offset;
    c64 sl{0.0, 0.0}, sq{0.0, 0.0}, tw{0.0, 0.0};
    for (int mm = c.n - 1; mm >= 1; --mm) {
        sl = sl + lq[mm];
        sq = sq + qq[mm];
        tw = tw + sl * sq;
    }
    const double delta = fabs(c.z_free - c.z_contact) / (c.n - 1);
    const double g = delta / (kPi * c.radius * c.radius);
    const c64 iden = cinv(c64{c.sigma, omega * p.eps});
    const c64 z = c64{0.0, g * omega} * iden;
    const c64 tz = tw * z;
    part[((size_t)f * p.n_cols + w) * 2 + 0] = (tz * iden).re;
    part[((size_t)f * p.n_cols + w) * 2 + 1] = 2.0 * tz.re / c.radius;
}

// K_ij = sum_f Re[lambda_i(w_f) q_j(w_f)].
__global__ void __launch_bounds__(kBlock) k_adj_outer(Plan p, const c64* qw, const c64* lam, double* K) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= p.n_q) return;
    double acc = 0.0;
    for (int f = 0; f < p.n_freq; ++f) {
        const c64 a = lam[(size_t)f * p.n + i], b = qw[(size_t)f * p.n + j];
        acc += a.re * b.re - a.im * b.im;
    }
    K[(size_t)i * p.n_q + j] = acc;
}

// Collocation-matrix terms: dA_ij/d(offset of row column) and dA_ij/d(width of
// source column), each times K_ij, from the lattice-sum derivative tables as
// the matrix itself is built from g.
__global__ void __launch_bounds__(kBlock) k_adj_dA(Plan p, const double* gd, const double* A, const double* K,
                                                   double* prod) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= p.n_q) return;
    const int w = column_of(p, i), v = column_of(p, j);
    const double u = (node_z(p.col[w], i - p.col[w].offset) - node_z(p.col[v], j - p.col[v].offset)) / p.L[2];
    const size_t table = (size_t)p.n_cols * p.n_cols * p.nkz_tab;
    const double* gx = gd + (size_t)(v * p.n_cols + w) * p.nkz_tab;
    const double* gs = gx + table;
    const double* gp = gs + table;
    double ax = 0.0, as = 0.0, ap = 0.0;
    for (int iz = p.col[v].mmax[2]; iz >= 1; --iz) {
        double t = iz * u;
        t -= rint(t);
        const double c = cospi(2.0 * t);
        ax += gx[iz] * c;
        as += gs[iz] * c;
        ap += gp[iz] * c;
    }
    const double inv = 1.0 / (p.eps * p.L[0] * p.L[1] * p.L[2]);
    const double kij = K[(size_t)i * p.n_q + j];
    const size_t nn = (size_t)p.n_q * p.n_q;
    prod[(size_t)i * p.n_q + j] = (gx[0] + 2.0 * ax) * inv * kij;
    prod[nn + (size_t)i * p.n_q + j] = kColWidthFraction * (gs[0] + 2.0 * as) * inv * kij;
    // pitch: the lattice-sum derivative and -2 A from the cell volume
    prod[2 * nn + (size_t)i * p.n_q + j] = ((gp[0] + 2.0 * ap) * inv - 2.0 * A[(size_t)i * p.n_q + j]) * kij;
}

// Final reduction, one block: out[w][0..3] = dL/d resistivity (0 past
// n_resistivity), out[w][4] = dL/d radius, out[5 n_cols] = dL/d pitch (per
// metre of L_x: the scale derivative divided by L_x).
__global__ void __launch_bounds__(kBlock) k_adj_params(Plan p, const double* part, const double* prod,
                                                       const double* pitch, double* out) {
    __shared__ double red[kBlock / 64];
    const int tid = threadIdx.x, nq = p.n_q, W = p.n_cols;
    const size_t nn = (size_t)nq * nq;
    for (int w = 0; w < W; ++w) {
        const Column& c = p.col[w];
        double s0 = 0.0, s1 = 0.0, sx = 0.0, ss = 0.0;
        for (int f = tid; f < p.n_freq; f += blockDim.x) {
            s0 += part[((size_t)f * W + w) * 2 + 0];
            s1 += part[((size_t)f * W + w) * 2 + 1];
        }
        for (int idx = tid; idx < c.n * nq; idx += blockDim.x) {      // rows of column w
            const int i = c.offset + idx / nq, j = idx % nq;
            sx += prod[(size_t)i * nq + j];
        }
        for (int idx = tid; idx < nq * c.n; idx += blockDim.x) {      // columns of column w
            const int i = idx / c.n, j = c.offset + idx % c.n;
            ss += prod[nn + (size_t)i * nq + j];
        }
        s0 = block_sum_all(s0, red);
        s1 = block_sum_all(s1, red);
        sx = block_sum_all(sx, red);
        ss = block_sum_all(ss, red);
        if (tid == 0) {
            for (int q = 0; q < 4; ++q)
                out[w * 5 + q] = q < c.n_res ? s0 * (-1.0 / (c.n_res * c.resistivity[q] * c.resistivity[q])) : 0.0;
            out[w * 5 + 4] = s1 - sx - ss;
        }
    }
    double sp = 0.0, sq = 0.0;
    for (size_t idx = tid; idx < nn; idx += blockDim.x) sp += prod[2 * nn + idx];
    for (int t = tid; t < p.n_time; t += blockDim.x) sq += pitch[t];
    sp = block_sum_all(sp, red);
    sq = block_sum_all(sq, red);
    if (tid == 0) out[W * 5] = (sq - sp) / p.L[0];
}

template <typename T>
hipError_t adjoint_rhs(const Plan& p, const GradLayout& g, const char* ws, int n_carriers, const T* pos,
                       const T* charge, const int* track, const T* grad_i, char* gws, hipStream_t s) {
    cplx<T>* phi = reinterpret_cast<cplx<T>*>(gws + g.off_phi);
    cplx<T>* phis = reinterpret_cast<cplx<T>*>(gws + g.off_phis);
    const int n_items = p.n_cols * p.nzh;
    const size_t n_phi = (size_t)g.n_tracks * p.n_time * n_items * 2;
    const int zgrid = (int)std::min<size_t>((n_phi + kBlock - 1) / kBlock, 4096);
    hipLaunchKernelGGL(k_adj_fill<T>, dim3(zgrid), dim3(kBlock), 0, s, reinterpret_cast<T*>(phi), n_phi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_fill<T>, dim3(zgrid), dim3(kBlock), 0, s, reinterpret_cast<T*>(phis), n_phi);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (n_carriers > 0) {
        const int chunk = std::max(64, (n_carriers + 65534) / 65535);
        dim3 grid(p.n_time, (n_carriers + chunk - 1) / chunk, (n_items + kBlock - 1) / kBlock);
        hipLaunchKernelGGL(k_adj_events<T>, grid, dim3(kBlock), 0, s, p,
                           reinterpret_cast<const cplx<T>*>(ws + p.off_ehat),
                           reinterpret_cast<const cplx<T>*>(gws + g.off_eds),
                           reinterpret_cast<const cplx<T>*>(ws + p.off_tw[2]), n_carriers, g.n_tracks, pos, charge,
                           track, chunk, phi, phis);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    c64* gamma = reinterpret_cast<c64*>(gws + g.off_gamma);
    hipLaunchKernelGGL(k_adj_gamma<T>, dim3((n_items + kBlock - 1) / kBlock, p.n_time), dim3(kBlock), 0, s, p,
                       g.n_tracks, (const cplx<T>*)phi, grad_i, gamma);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    c64* gammas = reinterpret_cast<c64*>(gws + g.off_gammas);
    hipLaunchKernelGGL(k_adj_gamma<T>, dim3((n_items + kBlock - 1) / kBlock, p.n_time), dim3(kBlock), 0, s, p,
                       g.n_tracks, (const cplx<T>*)phis, grad_i, gammas);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_pitch_lag<T>, dim3(p.n_time), dim3(kBlock), 0, s, p, (const c64*)gammas,
                       reinterpret_cast<const cplx<T>*>(ws + p.off_qhat), reinterpret_cast<double*>(gws + g.off_pitch));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double* gbar = reinterpret_cast<double*>(gws + g.off_gbar);
    hipLaunchKernelGGL(k_adj_sources, dim3((p.n_q + kBlock - 1) / kBlock, p.n_time), dim3(kBlock), 0, s, p,
                       (const c64*)gamma, gbar);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_rhs, dim3((p.n + kBlock - 1) / kBlock, p.n_freq), dim3(kBlock), 0, s, p,
                       (const double*)gbar, reinterpret_cast<c64*>(gws + g.off_rhs));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adjoint_rhs(const Plan& p, const GradLayout& g, const void* ws, int n_carriers, const void* pos,
                              const void* charge, const int* track, const void* grad_i, void* gws, hipStream_t s) {
    const char* b = static_cast<const char*>(ws);
    char* gb = static_cast<char*>(gws);
    if (p.precision == 0)
        return adjoint_rhs<double>(p, g, b, n_carriers, static_cast<const double*>(pos),
                                   static_cast<const double*>(charge), track, static_cast<const double*>(grad_i),
                                   gb, s);
    return adjoint_rhs<float>(p, g, b, n_carriers, static_cast<const float*>(pos), static_cast<const float*>(charge),
                              track, static_cast<const float*>(grad_i), gb, s);
}

hipError_t launch_adjoint_params(const Plan& p, const GradLayout& g, const void* ws, void* gws, double* out,
                                 hipStream_t s) {
    const char* b = static_cast<const char*>(ws);
    char* gb = static_cast<char*>(gws);
    const c64* qw = reinterpret_cast<const c64*>(b + p.off_qw);
    const c64* lam = reinterpret_cast<const c64*>(gb + g.off_lam);
    double* part = reinterpret_cast<double*>(gb + g.off_part);
    double* K = reinterpret_cast<double*>(gb + g.off_K);
    double* prod = reinterpret_cast<double*>(gb + g.off_prod);
    hipLaunchKernelGGL(k_adj_freq, dim3(p.n_freq), dim3(64), 0, s, p, qw, lam, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_outer, dim3((p.n_q + kBlock - 1) / kBlock, p.n_q), dim3(kBlock), 0, s, p, qw, lam, K);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_dA, dim3((p.n_q + kBlock - 1) / kBlock, p.n_q), dim3(kBlock), 0, s, p,
                       reinterpret_cast<const double*>(gb + g.off_gd), reinterpret_cast<const double*>(b + p.off_A),
                       (const double*)K, prod);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_params, dim3(1), dim3(kBlock), 0, s, p, (const double*)part, (const double*)prod,
                       reinterpret_cast<const double*>(gb + g.off_pitch), out);
    return hipGetLastError();
}

}  // namespace wt
