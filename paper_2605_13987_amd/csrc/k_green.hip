// Green's tables of the boundary fit (FP64) and FFT twiddle tables.
//
// The boundary fit uses the periodic fundamental solution of a Gaussian
// charge of width s_c = r/4 on the column axis (abstract: fundamental
// solutions impose the boundary conditions), as the converged Fourier series
//   G_c(d) = 1/(eps V) sum_{k != 0} exp(-k^2 s_c^2 / 2) cos(k.d) / k^2,
// k = 2 pi (m_x/L_x, m_y/L_y, m_z/L_z), |m_a| <= mmax_a (terms beyond are below
// exp(-40) of the leading ones).  A collocation point and a source of another
// (or the same) column are separated in-plane by one vector per column pair,
// so the sum is split: g_vw(k_z) = sum_{m_x, m_y} exp(-k^2 s_c^2/2) / k^2
// cos(k_x dx + k_y dy) once per pair and k_z >= 0 (g is even in k_z), then
// A_ij = 1/(eps V) [g(0) + 2 sum_{k_z > 0} g(k_z) cos(k_z (z_i - z_j))].
#include "common.hpp"

namespace wt {

namespace {

constexpr int kBlock = 256;

__device__ inline double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    }
    return s;   // valid in thread 0
}

template <typename T>
__global__ void k_twiddles(int n0, int n1, int n2, cplx<T>* t0, cplx<T>* t1, cplx<T>* t2) {
    const int axis = blockIdx.y;
    const int n = axis == 0 ? n0 : (axis == 1 ? n1 : n2);
    cplx<T>* t = axis == 0 ? t0 : (axis == 1 ? t1 : t2);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
        double s, c;
        sincospi(2.0 * (double)j / (double)n, &s, &c);
        t[j] = cplx<T>{(T)c, (T)s};      // exp(+2 pi i j / n)
    }
}

// One block per (k_z >= 0, source column v, collocation column w).  kind 0:
// g_vw(k_z); kind 1: its derivative in the in-plane offset dx (collocation
// column's radius), sum exp(-k^2 s^2/2)/k^2 (-k_x sin(k_x dx + k_y dy));
// kind 2: its derivative in the source width s, sum -s exp(-k^2 s^2/2)
// cos(k_x dx + k_y dy); kind 3: its derivative under a uniform scaling of the
// in-plane cell size and column positions by t (pitch), at t = 1: k_x, k_y
// scale as 1/t and the offset dx as (X_w - X_v) t + r, so with f =
// exp(-k^2 s^2/2)/k^2 the term is f (s^2 + 2/k^2)(k_x^2 + k_y^2) cos(k_x dx +
// k_y dy) + f k_x r sin(k_x dx + k_y dy).
// The in-plane sums factor along the axes except for 1/k^2: with
// exp(-k^2 s^2/2) = e_x(m_x) e_y(m_y) e_z and cos(2 pi (m_x a_x + m_y a_y))
// from the per-axis cosines and sines, one term costs a few products and a
// division instead of an exponential and a cosine.  The per-axis tables live
// in LDS (up to kMaxAxisModes modes per axis; wider mode boxes take the
// direct form).
constexpr int kMaxAxisModes = 1024;

__global__ void __launch_bounds__(kBlock) k_lattice(Plan p, int kind, double* g) {
    __shared__ double red[kBlock / 64];
    __shared__ double tx[3][kMaxAxisModes], ty[3][kMaxAxisModes];   // e, cos, sin per axis mode
    const int iz = blockIdx.x;
    const int v = blockIdx.y / p.n_cols, w = blockIdx.y % p.n_cols;
    const Column& cv = p.col[v];
    const Column& cw = p.col[w];
    double* out = g + (size_t)(v * p.n_cols + w) * p.nkz_tab;
    if (iz > cv.mmax[2]) {
        if (threadIdx.x == 0 && iz < p.nkz_tab) out[iz] = 0.0;
        return;
    }
    const double sc = cv.width;
    const double ax = (cw.x + cw.radius - cv.x) / p.L[0];
    const double ay = (cw.y - cv.y) / p.L[1];
    const double kz = 2.0 * kPi * iz / p.L[2];
    const int mx0 = cv.mmax[0], my0 = cv.mmax[1];
    const int nx = 2 * mx0 + 1, ny = 2 * my0 + 1;
    const int total = nx * ny;
    double acc = 0.0;
    if (nx <= kMaxAxisModes && ny <= kMaxAxisModes) {
        for (int i = threadIdx.x; i < nx + ny; i += blockDim.x) {
            const bool isx = i < nx;
            const int m = isx ? i - mx0 : i - nx - my0;
            const double k = 2.0 * kPi * m / (isx ? p.L[0] : p.L[1]);
            double u = m * (isx ? ax : ay);
            u -= rint(u);
            double sn, cs;
            sincospi(2.0 * u, &sn, &cs);
            double* t = isx ? &tx[0][i] : &ty[0][i - nx];
            t[0] = exp(-0.5 * k * k * sc * sc);
            t[kMaxAxisModes] = cs;
            t[2 * kMaxAxisModes] = sn;
        }
        __syncthreads();
        const double ez = exp(-0.5 * kz * kz * sc * sc);
        for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
            const int ix = idx / ny, iy = idx - (idx / ny) * ny;
            const int mx = ix - mx0, my = iy - my0;
            if (iz == 0 && mx == 0 && my == 0) continue;
            const double kx = 2.0 * kPi * mx / p.L[0];
            const double ky = 2.0 * kPi * my / p.L[1];
            const double k2 = kx * kx + ky * ky + kz * kz;
            const double e = ez * tx[0][ix] * ty[0][iy];
            const double c = tx[1][ix] * ty[1][iy] - tx[2][ix] * ty[2][iy];    // cos(2 pi (m_x a_x + m_y a_y))
            if (kind == 0) {
                acc += e / k2 * c;
            } else {
                const double sn = tx[2][ix] * ty[1][iy] + tx[1][ix] * ty[2][iy]; // sin(...)
                if (kind == 1)
                    acc -= e / k2 * kx * sn;
                else if (kind == 2)
                    acc -= sc * e * c;
                else
                    acc += e / k2 * ((sc * sc + 2.0 / k2) * (kx * kx + ky * ky) * c + kx * cw.radius * sn);
            }
        }
        const double sum = block_sum(acc, red);
        if (threadIdx.x == 0) out[iz] = sum;
        return;
    }
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
        const int mx = idx / ny - mx0;
        const int my = idx % ny - my0;
        if (iz == 0 && mx == 0 && my == 0) continue;
        const double kx = 2.0 * kPi * mx / p.L[0];
        const double ky = 2.0 * kPi * my / p.L[1];
        const double k2 = kx * kx + ky * ky + kz * kz;
        double u = mx * ax + my * ay;
        u -= rint(u);
        const double e = exp(-0.5 * k2 * sc * sc);
        if (kind == 0)
            acc += e / k2 * cospi(2.0 * u);
        else if (kind == 1)
            acc -= e / k2 * kx * sinpi(2.0 * u);
        else if (kind == 2)
            acc -= sc * e * cospi(2.0 * u);
        else
            acc += e / k2 * ((sc * sc + 2.0 / k2) * (kx * kx + ky * ky) * cospi(2.0 * u) + kx * cw.radius * sinpi(2.0 * u));
    }
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) out[iz] = s;
}

__device__ inline void node_of(const Plan& p, int i, int& col, int& m) {
    col = 0;
    while (col + 1 < p.n_cols && i >= p.col[col + 1].offset) ++col;
    m = i - p.col[col].offset;
}

__device__ inline double node_z(const Column& c, int m) {
    return c.z_contact + (m * (c.z_free - c.z_contact)) / (c.n - 1);
}

// A[i][j] = G_c(x_i - y_j): i collocation node (row), j source node (column).
__global__ void __launch_bounds__(kBlock) k_collocation_matrix(Plan p, const double* g, double* A) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int i = blockIdx.y;
    if (j >= p.n_q) return;
    int w, mi, v, mj;
    node_of(p, i, w, mi);
    node_of(p, j, v, mj);
    const double u = (node_z(p.col[w], mi) - node_z(p.col[v], mj)) / p.L[2];
    const double* gr = g + (size_t)(v * p.n_cols + w) * p.nkz_tab;
    double acc = 0.0;
    for (int iz = p.col[v].mmax[2]; iz >= 1; --iz) {
        double t = iz * u;
        t -= rint(t);
        acc += gr[iz] * cospi(2.0 * t);
    }
    acc = gr[0] + 2.0 * acc;
    const double vol = p.L[0] * p.L[1] * p.L[2];
    A[(size_t)i * p.n_q + j] = acc / (p.eps * vol);
}

}  // namespace

hipError_t launch_twiddles(const Plan& p, void* ws, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    const int nmax = p.N[0] > p.N[1] ? (p.N[0] > p.N[2] ? p.N[0] : p.N[2]) : (p.N[1] > p.N[2] ? p.N[1] : p.N[2]);
    dim3 grid((nmax + kBlock - 1) / kBlock, 3);
    if (p.precision == 0) {
        hipLaunchKernelGGL(k_twiddles<double>, grid, dim3(kBlock), 0, s, p.N[0], p.N[1], p.N[2],
                           (cplx<double>*)(b + p.off_tw[0]), (cplx<double>*)(b + p.off_tw[1]),
                           (cplx<double>*)(b + p.off_tw[2]));
    } else {
        hipLaunchKernelGGL(k_twiddles<float>, grid, dim3(kBlock), 0, s, p.N[0], p.N[1], p.N[2],
                           (cplx<float>*)(b + p.off_tw[0]), (cplx<float>*)(b + p.off_tw[1]),
                           (cplx<float>*)(b + p.off_tw[2]));
    }
    return hipGetLastError();
}

hipError_t launch_green_tables(const Plan& p, void* ws, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    double* g = (double*)(b + p.off_g);
    double* A = (double*)(b + p.off_A);
    hipLaunchKernelGGL(k_lattice, dim3(p.nkz_tab, p.n_cols * p.n_cols), dim3(kBlock), 0, s, p, 0, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_collocation_matrix, dim3((p.n_q + kBlock - 1) / kBlock, p.n_q), dim3(kBlock), 0, s,
                       p, (const double*)g, A);
    return hipGetLastError();
}

hipError_t launch_lattice_derivatives(const Plan& p, double* gd, hipStream_t s) {
    const size_t table = (size_t)p.n_cols * p.n_cols * p.nkz_tab;
    for (int kind = 1; kind <= 3; ++kind) {
        hipLaunchKernelGGL(k_lattice, dim3(p.nkz_tab, p.n_cols * p.n_cols), dim3(kBlock), 0, s, p, kind,
                           gd + (kind - 1) * table);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace wt
