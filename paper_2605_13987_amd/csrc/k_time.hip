// Frequency-to-time transform of the source charges and their per-column
// z-transform.
//
// The field is linear in the charges, so transforming the charges instead of
// the field gives the same H(x, t_n) (convention exp(+i w t), real response):
//   q_i(t_n) = df sum_j c_j Re[q_i(w_j) exp(+2 pi i j n df dt)]
// with c_0 = 1, c_j = 2 inside the band and c_last = 1 when the last
// frequency is 1/(2 dt).  Then, per column w and k_z = 2 pi m_z / L_z with
// 0 <= m_z < N_z/2,
//   Qhat_w(m_z, t_n) = sum_m q_{w,m}(t_n) exp(-i k_z z_{w,m}).
#include "common.hpp"

namespace wt {

namespace {

constexpr int kBlock = 256;

__global__ void __launch_bounds__(kBlock) k_charges_in_time(Plan p, const cplx<double>* qw, double* qt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = blockIdx.y;
    if (i >= p.n_q) return;
    const double r = p.df * p.dt;
    double acc = 0.0;
    for (int j = 0; j < p.n_freq; ++j) {
        const double cj = (j == 0 || (j == p.n_freq - 1 && p.last_weight_one)) ? 1.0 : 2.0;
        double x = (double)((long long)j * nt) * r;
        x -= floor(x);
        double s, c;
        sincospi(2.0 * x, &s, &c);
        const cplx<double> q = qw[(size_t)j * p.n + i];
        acc += cj * (q.re * c - q.im * s);
    }
    qt[(size_t)nt * p.n_q + i] = acc * p.df;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_column_ztransform(Plan p, const double* qt, cplx<T>* qhat) {
    const int mz = blockIdx.x * blockDim.x + threadIdx.x;
    const int nt = blockIdx.y;
    const int w = blockIdx.z;
    if (mz >= p.nzh) return;
    const Column& c = p.col[w];
    const double* q = qt + (size_t)nt * p.n_q + c.offset;
    double re = 0.0, im = 0.0;
    for (int m = 0; m < c.n; ++m) {
        const double z = c.z_contact + (m * (c.z_free - c.z_contact)) / (c.n - 1);
        double x = mz * (z / p.L[2]);
        x -= floor(x);
        double s, cs;
        sincospi(2.0 * x, &s, &cs);
        re += q[m] * cs;
        im -= q[m] * s;
    }
    qhat[((size_t)nt * p.n_cols + w) * p.nzh + mz] = cplx<T>{(T)re, (T)im};
}

}  // namespace

hipError_t launch_time_transform(const Plan& p, void* ws, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    const cplx<double>* qw = (const cplx<double>*)(b + p.off_qw);
    double* qt = (double*)(b + p.off_qt);
    hipLaunchKernelGGL(k_charges_in_time, dim3((p.n_q + kBlock - 1) / kBlock, p.n_time), dim3(kBlock), 0, s,
                       p, qw, qt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((p.nzh + kBlock - 1) / kBlock, p.n_time, p.n_cols);
    if (p.precision == 0)
        hipLaunchKernelGGL(k_column_ztransform<double>, grid, dim3(kBlock), 0, s, p, (const double*)qt,
                           (cplx<double>*)(b + p.off_qhat));
    else
        hipLaunchKernelGGL(k_column_ztransform<float>, grid, dim3(kBlock), 0, s, p, (const double*)qt,
                           (cplx<float>*)(b + p.off_qhat));
    return hipGetLastError();
}

}  // namespace wt
