// Fundamental-solution boundary fit: one bordered complex system per
// frequency, solved in FP64 by LU with partial pivoting and refined with an
// FP64 residual (paper, abstract and Section 3: point charges at the
// electrode boundaries whose magnitudes enforce the boundary conditions).
//
// Unknowns q (column node charges, C/V) and the gauge c.  For node i = (w,m):
//   sum_j A_ij q_j + i w sum_{m'} R_w(min(m, m')) q_{w,m'} + c = V_app(w)
//   sum_j q_j = 0
// with R_w(m) = m D_w / (pi r_w^2 (sigma_w + i w eps)) the cumulative
// resistance of the column's RC line (contact node m = 0 at V_app).  The
// system is equilibrated: unknowns q' = a q with a = max |A_ii| and the
// neutrality row multiplied by a, so that every block is of order one.
//
// One workgroup per frequency; n_q <= 128 factors the source block in
// registers (Schur complement of the gauge border), n <= 144 the bordered
// system in registers, larger systems in the workspace by blocks of 16
// columns; the matrix entries are regenerated from A for the refinement
// residual.
#include "common.hpp"

#include <algorithm>

namespace wt {

namespace {

constexpr int kMaxN = 528;

using c64 = cplx<double>;

__device__ inline double cabs1(c64 a) { return fabs(a.re) + fabs(a.im); }
__device__ inline double cmod(c64 a) { return sqrt(a.re * a.re + a.im * a.im); }

__device__ inline c64 cinv(c64 a) {
    const double d = a.re * a.re + a.im * a.im;
    return d == 0.0 ? c64{0.0, 0.0} : c64{a.re / d, -a.im / d};
}

struct NodeMap {
    int col;
    int m;
};

__device__ inline NodeMap node_of(const Plan& p, int i) {
    int col = 0;
    while (col + 1 < p.n_cols && i >= p.col[col + 1].offset) ++col;
    return NodeMap{col, i - p.col[col].offset};
}

// Entry (i, j) of the equilibrated system matrix.
__device__ inline c64 s_entry(const Plan& p, const double* A, double inv_a, const c64* zc, int i, int j) {
    const int nq = p.n_q;
    if (i < nq && j < nq) {
        c64 v{A[(size_t)i * nq + j], 0.0};
        const NodeMap a = node_of(p, i), b = node_of(p, j);
        if (a.col == b.col) {
            const double mm = (double)(a.m < b.m ? a.m : b.m);
            v = v + scale(zc[a.col], mm);
        }
        return scale(v, inv_a);
    }
    if (i == nq && j == nq) return c64{0.0, 0.0};
    return c64{1.0, 0.0};
}

__device__ inline double block_max(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) s = fmax(s, red[i]);
    return s;   // valid in every thread
}

__device__ inline c64 block_csum(c64 v, c64* red) {
    for (int o = 32; o > 0; o >>= 1) {
        v.re += __shfl_xor(v.re, o, 64);
        v.im += __shfl_xor(v.im, o, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    c64 s = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) s = s + red[i];
    return s;   // valid in every thread
}

// x <- (LU)^-1 P x, with LU and the pivots of one frequency.
__device__ void lu_solve(int n, const c64* lu, const int* piv, c64* x) {
    const int tid = threadIdx.x;
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < n; ++k) {
            const int q = piv[k];
            if (q != k) {
                const c64 t = x[k];
                x[k] = x[q];
                x[q] = t;
            }
        }
    }
    __syncthreads();
    for (int k = 0; k < n - 1; ++k) {            // unit lower triangle
        const c64 yk = x[k];
        for (int i = k + 1 + tid; i < n; i += blockDim.x) x[i] = x[i] - lu[(size_t)i * n + k] * yk;
        __syncthreads();
    }
    for (int k = n - 1; k >= 0; --k) {           // upper triangle
        if (tid == 0) x[k] = x[k] * cinv(lu[(size_t)k * n + k]);
        __syncthreads();
        const c64 yk = x[k];
        for (int i = tid; i < k; i += blockDim.x) x[i] = x[i] - lu[(size_t)i * n + k] * yk;
        __syncthreads();
    }
}

// Solve with the LU factors, refine with the FP64 residual of the
// equilibrated system, and store the charges and the report of frequency f.
__device__ void refine_and_store(const Plan& p, const double* A, double inv_a, const c64* zc, const c64* lu,
                                 const int* pivs, c64* xs, c64* rs, double* red, int f, c64* qw,
                                 SolveReport* rep, double umax, double umin, int singular) {
    const int n = p.n, nq = p.n_q, tid = threadIdx.x;
    // right-hand side: applied voltages, 0 for the neutrality row
    for (int i = tid; i < n; i += blockDim.x) {
        c64 b{0.0, 0.0};
        if (i < nq) b.re = p.col[node_of(p, i).col].v_applied;
        xs[i] = b;
    }
    lu_solve(n, lu, pivs, xs);

    // infinity norms of S and b
    double srow = 0.0, bmax = 0.0;
    for (int i = tid; i < n; i += blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < n; ++j) s += cmod(s_entry(p, A, inv_a, zc, i, j));
        srow = fmax(srow, s);
        if (i < nq) bmax = fmax(bmax, fabs(p.col[node_of(p, i).col].v_applied));
    }
    const double snorm = block_max(srow, red);
    const double bnorm = block_max(bmax, red);

    int iters = 0;
    double berr = 0.0;
    for (;;) {
        double rmax = 0.0, xmax = 0.0;
        for (int i = tid; i < n; i += blockDim.x) {
            c64 acc{0.0, 0.0};
            if (i < nq) acc.re = p.col[node_of(p, i).col].v_applied;
            for (int j = 0; j < n; ++j) acc = acc - s_entry(p, A, inv_a, zc, i, j) * xs[j];
            rs[i] = acc;
            rmax = fmax(rmax, cmod(acc));
            xmax = fmax(xmax, cmod(xs[i]));
        }
        rmax = block_max(rmax, red);
        xmax = block_max(xmax, red);
        const double den = snorm * xmax + bnorm;
        berr = den > 0.0 ? rmax / den : 0.0;
        if (berr <= p.ir_tol || iters >= p.ir_max_iter) break;
        lu_solve(n, lu, pivs, rs);
        for (int i = tid; i < n; i += blockDim.x) xs[i] = xs[i] + rs[i];
        __syncthreads();
        ++iters;
    }

    for (int i = tid; i < n; i += blockDim.x) {
        const c64 v = xs[i];
        qw[(size_t)f * n + i] = i < nq ? scale(v, inv_a) : v;
    }
    if (tid == 0) {
        rep[f].backward_error = berr;
        rep[f].pivot_ratio = umin > 0.0 ? umax / umin : 1e308;
        rep[f].iters = iters;
        rep[f].singular = singular;
    }
}

// Blocked right-looking factorisation for any n <= kMaxN, one workgroup per
// frequency, the matrix in the workspace.  Per panel of NB columns:
//  1. the panel (rows k0..n-1) is factored in LDS with partial pivoting;
//  2. its row interchanges are applied to the columns left and right of it;
//  3. the block row right of it becomes U12 = L11^-1 A12 (unit lower solve);
//  4. the trailing matrix is updated once, A22 -= L21 U12, with L21 read from
//     LDS: every element of A22 is read and written once per panel instead of
//     once per column, which divides the HBM traffic of the factorisation by NB.
// The factors and the interchanges are those of the unblocked algorithm (same
// pivot rule: first row of maximal |re| + |im|), so the refinement's
// triangular solves are unchanged.
constexpr int kPanel = 16;
constexpr int kBlockedThreads = 1024;

__global__ void __launch_bounds__(kBlockedThreads)
k_solve_blocked(Plan p, const double* A, c64* lu_all, int* piv_all, c64* qw, SolveReport* rep) {
    extern __shared__ __align__(16) unsigned char smem[];
    c64* panel = reinterpret_cast<c64*>(smem);            // [n - k0][kPanel], row-major
    __shared__ int pivs[kMaxN];
    __shared__ c64 zc[kMaxCols];
    __shared__ double red[kBlockedThreads / 64];
    __shared__ int red_i[kBlockedThreads / 64];
    __shared__ double red_v[kBlockedThreads / 64];
    __shared__ double sh_inv_a;
    __shared__ int sh_piv;
    __shared__ int sh_singular;

    const int f = blockIdx.x;
    const int n = p.n, nq = p.n_q, tid = threadIdx.x, nth = blockDim.x;
    const double omega = 2.0 * kPi * p.df * f;
    c64* lu = lu_all + (size_t)f * n * n;
    int* piv = piv_all + (size_t)f * n;

    if (tid < p.n_cols) {
        const Column& c = p.col[tid];
        const double delta = fabs(c.z_free - c.z_contact) / (c.n - 1);
        const double g = delta / (kPi * c.radius * c.radius);
        const double den = c.sigma * c.sigma + omega * omega * p.eps * p.eps;
        zc[tid] = c64{g * omega * omega * p.eps / den, g * omega * c.sigma / den};
    }
    double dmax = 0.0;
    for (int i = tid; i < nq; i += nth) dmax = fmax(dmax, fabs(A[(size_t)i * nq + i]));
    dmax = block_max(dmax, red);
    if (tid == 0) {
        sh_inv_a = 1.0 / dmax;
        sh_singular = 0;
    }
    __syncthreads();
    const double inv_a = sh_inv_a;
    for (int idx = tid; idx < n * n; idx += nth) lu[idx] = s_entry(p, A, inv_a, zc, idx / n, idx % n);
    __syncthreads();

    double umax = 0.0, umin = 1e308;
    for (int k0 = 0; k0 < n; k0 += kPanel) {
        const int nb = min(kPanel, n - k0);
        const int mp = n - k0;
        // 1. panel into LDS and factored there
        for (int idx = tid; idx < mp * nb; idx += nth) {
            const int r = idx / nb, c = idx - (idx / nb) * nb;
            panel[r * kPanel + c] = lu[(size_t)(k0 + r) * n + k0 + c];
        }
        __syncthreads();
        for (int c = 0; c < nb; ++c) {
            double best = -1.0;
            int bi = mp;
            for (int r = c + tid; r < mp; r += nth) {
                const double v = cabs1(panel[r * kPanel + c]);
                if (v > best) { best = v; bi = r; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_down(best, o, 64);
                const int oi = __shfl_down(bi, o, 64);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if ((tid & 63) == 0) { red_v[tid >> 6] = best; red_i[tid >> 6] = bi; }
            __syncthreads();
            if (tid == 0) {
                double bv = red_v[0];
                int b = red_i[0];
                for (int w = 1; w < nth / 64; ++w)
                    if (red_v[w] > bv || (red_v[w] == bv && red_i[w] < b)) { bv = red_v[w]; b = red_i[w]; }
                sh_piv = b;
                pivs[k0 + c] = k0 + b;
                piv[k0 + c] = k0 + b;
                if (!(bv > 0.0)) sh_singular = 1;
            }
            __syncthreads();
            const int pr = sh_piv;
            if (pr != c && tid < nb) {
                const c64 t = panel[c * kPanel + tid];
                panel[c * kPanel + tid] = panel[pr * kPanel + tid];
                panel[pr * kPanel + tid] = t;
            }
            __syncthreads();
            const c64 pivot = panel[c * kPanel + c];
            const double pm = cmod(pivot);
            umax = fmax(umax, pm);
            umin = fmin(umin, pm);
            const c64 ip = cinv(pivot);
            for (int r = c + 1 + tid; r < mp; r += nth) {
                c64* row = panel + r * kPanel;
                const c64 l = row[c] * ip;
                row[c] = l;
                for (int cc = c + 1; cc < nb; ++cc) row[cc] = row[cc] - l * panel[c * kPanel + cc];
            }
            __syncthreads();
        }
        for (int idx = tid; idx < mp * nb; idx += nth) {
            const int r = idx / nb, c = idx - (idx / nb) * nb;
            lu[(size_t)(k0 + r) * n + k0 + c] = panel[r * kPanel + c];
        }
        // 2. the panel's interchanges on the other columns (in order)
        for (int c = 0; c < nb; ++c) {
            const int r1 = k0 + c, r2 = pivs[k0 + c];
            if (r2 == r1) continue;
            for (int j = tid; j < n - nb; j += nth) {
                const int col = j < k0 ? j : j + nb;
                const c64 t = lu[(size_t)r1 * n + col];
                lu[(size_t)r1 * n + col] = lu[(size_t)r2 * n + col];
                lu[(size_t)r2 * n + col] = t;
            }
            __syncthreads();
        }
        __syncthreads();
        const int nr = n - k0 - nb;                       // columns (and rows) right of / below the panel
        if (nr > 0) {
            // 3. U12 = L11^-1 A12, one column per thread
            for (int j = k0 + nb + tid; j < n; j += nth) {
                c64* uj = lu + (size_t)k0 * n + j;
                for (int r = 1; r < nb; ++r) {
                    c64 acc = uj[(size_t)r * n];
                    for (int c = 0; c < r; ++c) acc = acc - panel[r * kPanel + c] * uj[(size_t)c * n];
                    uj[(size_t)r * n] = acc;
                }
            }
            __syncthreads();
            // 4. A22 -= L21 U12: each thread a 2 x 4 tile of A22 (4 consecutive columns)
            const int tcols = (nr + 3) / 4, trows = (nr + 1) / 2;
            for (int t = tid; t < tcols * trows; t += nth) {
                const int tc = t % tcols, tr = t / tcols;
                const int i0 = k0 + nb + 2 * tr, j0 = k0 + nb + 4 * tc;
                c64 acc[2][4];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = c64{0.0, 0.0};
                for (int c = 0; c < nb; ++c) {
                    c64 uv[4];
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        uv[b] = j0 + b < n ? lu[(size_t)(k0 + c) * n + j0 + b] : c64{0.0, 0.0};
#pragma unroll
                    for (int a = 0; a < 2; ++a) {
                        const c64 l = i0 + a < n ? panel[(i0 + a - k0) * kPanel + c] : c64{0.0, 0.0};
#pragma unroll
                        for (int b = 0; b < 4; ++b) acc[a][b] = acc[a][b] + l * uv[b];
                    }
                }
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b)
                        if (i0 + a < n && j0 + b < n) {
                            c64* e = lu + (size_t)(i0 + a) * n + j0 + b;
                            *e = *e - acc[a][b];
                        }
            }
        }
        __syncthreads();
    }

    // the panel's LDS holds the refinement vectors from here on
    c64* xs = panel;
    c64* rs = panel + kMaxN;
    refine_and_store(p, A, inv_a, zc, lu, pivs, xs, rs, red, f, qw, rep, umax, umin, sh_singular);
}

// Register-resident factorisation: TR x 32 threads, thread (r, c) holding rows
// r + TR ii (ii < NBR) and columns c + 32 jj (jj < NBC), so n <= min(TR NBR,
// 32 NBC).  Per pivot step: the TR owners of column k find the pivot (a
// reduction inside their wavefront), the two affected rows are exchanged
// through LDS, the pivot row and the multipliers are published in LDS, and
// every thread updates its block.  The factors are then written to the
// workspace for the triangular solves of the refinement.
template <int TR, int NBR, int NBC>
__global__ void __launch_bounds__(TR * 32)
k_solve_reg(Plan p, const double* A, c64* lu_all, int* piv_all, c64* qw, SolveReport* rep) {
    constexpr int NMAX = 32 * NBC;
    __shared__ c64 ubuf[NMAX];
    __shared__ c64 lbuf[TR * NBR];
    __shared__ c64 row_k[NMAX];
    __shared__ c64 row_p[NMAX];
    __shared__ c64 xs[kMaxN];
    __shared__ c64 rs[kMaxN];
    __shared__ int pivs[kMaxN];
    __shared__ c64 zc[kMaxCols];
    __shared__ double red[16];
    __shared__ double sh_inv_a;
    __shared__ int sh_piv;
    __shared__ double sh_pval;
    __shared__ int sh_singular;

    const int f = blockIdx.x;
    const int n = p.n, nq = p.n_q, tid = threadIdx.x;
    const int r = tid % TR, c = tid / TR;
    const double omega = 2.0 * kPi * p.df * f;
    c64* lu = lu_all + (size_t)f * n * n;
    int* piv = piv_all + (size_t)f * n;

    if (tid < p.n_cols) {
        const Column& cl = p.col[tid];
        const double delta = fabs(cl.z_free - cl.z_contact) / (cl.n - 1);
        const double g = delta / (kPi * cl.radius * cl.radius);
        const double den = cl.sigma * cl.sigma + omega * omega * p.eps * p.eps;
        zc[tid] = c64{g * omega * omega * p.eps / den, g * omega * cl.sigma / den};
    }
    double dmax = 0.0;
    for (int i = tid; i < nq; i += blockDim.x) dmax = fmax(dmax, fabs(A[(size_t)i * nq + i]));
    dmax = block_max(dmax, red);
    if (tid == 0) {
        sh_inv_a = 1.0 / dmax;
        sh_singular = 0;
    }
    __syncthreads();
    const double inv_a = sh_inv_a;

    c64 a[NBR][NBC];
#pragma unroll
    for (int ii = 0; ii < NBR; ++ii)
#pragma unroll
        for (int jj = 0; jj < NBC; ++jj) {
            const int i = r + TR * ii, j = c + 32 * jj;
            a[ii][jj] = (i < n && j < n) ? s_entry(p, A, inv_a, zc, i, j) : c64{0.0, 0.0};
        }

    double umax = 0.0, umin = 1e308;
    for (int k = 0; k < n; ++k) {
        const int kc = k & 31, kcq = k >> 5;         // owner column thread and its local column
        const int kr = k % TR, krq = k / TR;         // owner row thread and its local row
        if (c == kc) {                               // pivot search in column k
            double best = -1.0;
            int bi = n;
#pragma unroll
            for (int ii = 0; ii < NBR; ++ii) {
                const int i = r + TR * ii;
                c64 v = a[ii][0];
#pragma unroll
                for (int t = 1; t < NBC; ++t) if (kcq == t) v = a[ii][t];
                if (i >= k && i < n) {
                    const double m = cabs1(v);
                    if (m > best) { best = m; bi = i; }
                }
            }
            for (int o = TR / 2; o > 0; o >>= 1) {
                const double ov = __shfl_xor(best, o, TR);
                const int oi = __shfl_xor(bi, o, TR);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if (r == 0) {
                sh_piv = bi;
                sh_pval = best;
            }
        }
        __syncthreads();
        const int pr = sh_piv;
        if (tid == 0) {
            piv[k] = pr;
            pivs[k] = pr;
            if (!(sh_pval > 0.0)) sh_singular = 1;
        }
        if (pr != k) {                               // exchange rows k and pr through LDS
            const int pr_r = pr % TR, pr_q = pr / TR;
            if (r == kr || r == pr_r) {
#pragma unroll
                for (int jj = 0; jj < NBC; ++jj) {
                    const int j = c + 32 * jj;
                    c64 vk = a[0][jj], vp = a[0][jj];
#pragma unroll
                    for (int t = 1; t < NBR; ++t) {
                        if (krq == t) vk = a[t][jj];
                        if (pr_q == t) vp = a[t][jj];
                    }
                    if (j < n) {
                        if (r == kr) row_k[j] = vk;
                        if (r == pr_r) row_p[j] = vp;
                    }
                }
            }
            __syncthreads();
            if (r == kr || r == pr_r) {
#pragma unroll
                for (int jj = 0; jj < NBC; ++jj) {
                    const int j = c + 32 * jj;
                    if (j >= n) continue;
                    const c64 nk = row_p[j], np = row_k[j];
#pragma unroll
                    for (int t = 0; t < NBR; ++t) {
                        if (r == kr && krq == t) a[t][jj] = nk;
                        if (r == pr_r && pr_q == t) a[t][jj] = np;
                    }
                }
            }
        }
        if (r == kr) {                               // publish the pivot row (columns >= k)
#pragma unroll
            for (int jj = 0; jj < NBC; ++jj) {
                const int j = c + 32 * jj;
                c64 v = a[0][jj];
#pragma unroll
                for (int t = 1; t < NBR; ++t) if (krq == t) v = a[t][jj];
                if (j >= k && j < n) ubuf[j] = v;
            }
        }
        __syncthreads();
        const c64 pivot = ubuf[k];
        const double pm = cmod(pivot);
        umax = fmax(umax, pm);
        umin = fmin(umin, pm);
        const c64 ip = cinv(pivot);
        if (c == kc) {                               // multipliers of column k
#pragma unroll
            for (int ii = 0; ii < NBR; ++ii) {
                const int i = r + TR * ii;
                c64 v = a[ii][0];
#pragma unroll
                for (int t = 1; t < NBC; ++t) if (kcq == t) v = a[ii][t];
                const c64 l = v * ip;
                if (i > k && i < n) {
#pragma unroll
                    for (int t = 0; t < NBC; ++t) if (kcq == t) a[ii][t] = l;
                    lbuf[i] = l;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < NBR; ++ii) {
            const int i = r + TR * ii;
            if (i <= k || i >= n) continue;
            const c64 l = lbuf[i];
#pragma unroll
            for (int jj = 0; jj < NBC; ++jj) {
                const int j = c + 32 * jj;
                if (j > k && j < n) a[ii][jj] = a[ii][jj] - l * ubuf[j];
            }
        }
    }
#pragma unroll
    for (int ii = 0; ii < NBR; ++ii)
#pragma unroll
        for (int jj = 0; jj < NBC; ++jj) {
            const int i = r + TR * ii, j = c + 32 * jj;
            if (i < n && j < n) lu[(size_t)i * n + j] = a[ii][jj];
        }
    __syncthreads();
    refine_and_store(p, A, inv_a, zc, lu, pivs, xs, rs, red, f, qw, rep, umax, umin, sh_singular);
}

// y1 <- St^-1 y1 (and y2 <- St^-1 y2 when two), right-hand sides already
// permuted, with the factors held in registers by the 32 x 32 thread grid.
template <int NB>
__device__ __forceinline__ void solve_in_registers(const c64 (&a)[NB][NB], int m, int r, int cc, const c64* diag,
                                                   c64* y1, c64* y2, bool two) {
#pragma unroll
    for (int kq = 0; kq < NB; ++kq)                        // unit lower triangle
    for (int k32 = 0; k32 < 32; ++k32) {
        const int k = 32 * kq + k32;
        if (k >= m - 1) break;
        __syncthreads();
        if (cc == k32) {
            const c64 b1 = y1[k], b2 = two ? y2[k] : c64{0.0, 0.0};
#pragma unroll
            for (int ii = 0; ii < NB; ++ii) {
                const int i = r + 32 * ii;
                if (i > k && i < m) {
                    const c64 l = a[ii][kq];
                    y1[i] = y1[i] - l * b1;
                    if (two) y2[i] = y2[i] - l * b2;
                }
            }
        }
    }
#pragma unroll
    for (int kq = NB - 1; kq >= 0; --kq)                   // upper triangle
    for (int k32 = 31; k32 >= 0; --k32) {
        const int k = 32 * kq + k32;
        if (k >= m) continue;
        __syncthreads();
        if (cc == k32) {
            const c64 id = cinv(diag[k]);
            const c64 b1 = y1[k] * id, b2 = two ? y2[k] * id : c64{0.0, 0.0};
#pragma unroll
            for (int ii = 0; ii < NB; ++ii) {
                const int i = r + 32 * ii;
                if (i < k) {
                    const c64 u = a[ii][kq];
                    y1[i] = y1[i] - u * b1;
                    if (two) y2[i] = y2[i] - u * b2;
                }
            }
            if (r == k32) {           // owner of row k; its half-wavefront read y1[k] above
                y1[k] = b1;
                if (two) y2[k] = b2;
            }
        }
    }
    __syncthreads();
}

// Schur-complement form for n_q <= 32 NB: only the n_q x n_q block
// St = (A + i w R) / a is factored; with St x1 = b and St x2 = 1 the bordered
// system gives c = (1'x1) / (1'x2) and q' = x1 - c x2 (exact in exact
// arithmetic).  ADJ: the transposed system of the adjoint, S^T [l; c] =
// [rhs; 0] with rhs per frequency from the workspace; R is symmetric and the
// border is the same row and column of ones, so only A is read transposed.  1024 threads in a 32 x 32 grid, thread (r, c) holding rows
// r + 32 ii and columns c + 32 jj of St; the factors stay in registers for
// the triangular solves (one barrier per step: the owners of column k update
// the rows below or above k).  Refinement uses the residual of the bordered
// system, computed with one wavefront per row (coalesced reads of A).
template <int NB, bool ADJ>
__global__ void __launch_bounds__(1024)
k_solve_schur(Plan p, const double* A, const c64* rhs, c64* qw, SolveReport* rep) {
    constexpr int NM = 32 * NB;
    static_assert(NM <= 256, "the pivot key holds the row in 8 bits");
    __shared__ c64 ubuf[NM];
    __shared__ c64 lbuf[NM];
    __shared__ c64 row_k[NM];
    __shared__ c64 row_p[NM];
    __shared__ c64 diag[NM];
    __shared__ c64 y1[NM];
    __shared__ c64 y2[NM];
    __shared__ c64 xq[NM];
    __shared__ c64 rr[NM];
    __shared__ int perm[NM];
    __shared__ int pivs[NM];
    __shared__ unsigned char colof[NM];
    __shared__ short mof[NM];
    __shared__ c64 zc[kMaxCols];
    __shared__ double vapp[kMaxCols];
    __shared__ double red[16];
    __shared__ c64 redc[16];
    __shared__ double sh_inv_a;
    __shared__ int sh_piv;
    __shared__ double sh_pval;
    __shared__ int sh_singular;
    __shared__ c64 sh_c;

    const int f = blockIdx.x;
    const int m = p.n_q, tid = threadIdx.x;
    const int r = tid & 31, cc = tid >> 5;
    const int lane = tid & 63, wave = tid >> 6, nwave = blockDim.x >> 6;
    const double omega = 2.0 * kPi * p.df * f;

    if (tid < p.n_cols) {
        const Column& cl = p.col[tid];
        const double delta = fabs(cl.z_free - cl.z_contact) / (cl.n - 1);
        const double g = delta / (kPi * cl.radius * cl.radius);
        const double den = cl.sigma * cl.sigma + omega * omega * p.eps * p.eps;
        zc[tid] = c64{g * omega * omega * p.eps / den, g * omega * cl.sigma / den};
        vapp[tid] = cl.v_applied;
    }
    for (int i = tid; i < m; i += blockDim.x) {
        const NodeMap nm = node_of(p, i);
        colof[i] = (unsigned char)nm.col;
        mof[i] = (short)nm.m;
    }
    double dmax = 0.0;
    for (int i = tid; i < m; i += blockDim.x) dmax = fmax(dmax, fabs(A[(size_t)i * m + i]));
    dmax = block_max(dmax, red);
    if (tid == 0) {
        sh_inv_a = 1.0 / dmax;
        sh_singular = 0;
    }
    __syncthreads();
    const double inv_a = sh_inv_a;
    auto st = [&](int i, int j) -> c64 {                 // entry of St (of St^T for ADJ)
        c64 v{ADJ ? A[(size_t)j * m + i] : A[(size_t)i * m + j], 0.0};
        if (colof[i] == colof[j]) v = v + scale(zc[colof[i]], (double)(mof[i] < mof[j] ? mof[i] : mof[j]));
        return scale(v, inv_a);
    };

    c64 a[NB][NB];
#pragma unroll
    for (int ii = 0; ii < NB; ++ii)
#pragma unroll
        for (int jj = 0; jj < NB; ++jj) {
            const int i = r + 32 * ii, j = cc + 32 * jj;
            a[ii][jj] = (i < m && j < m) ? st(i, j) : c64{0.0, 0.0};
        }

#pragma unroll
    for (int kq = 0; kq < NB; ++kq)                        // local index of column k: compile-time
    for (int k32 = 0; k32 < 32; ++k32) {
        const int k = 32 * kq + k32;
        if (k >= m) break;
        if (cc == k32) {                                   // pivot search in column k
            // One 32-bit key per candidate: the high word of |re| + |im|
            // (exponent and 20 mantissa bits) with its low 8 bits replaced by
            // 255 - row.  One integer maximum (one shuffle per step) then
            // picks the largest magnitude to 12 mantissa bits and, among
            // magnitudes that agree that far, the first row.
            unsigned key = 0u;
#pragma unroll
            for (int ii = 0; ii < NB; ++ii) {
                const int i = r + 32 * ii;
                const c64 v = a[ii][kq];
                if (i >= k && i < m) {
                    const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(cabs1(v)) >> 32);
                    key = max(key, (hi & ~255u) | (unsigned)(255 - i));
                }
            }
            for (int o = 16; o > 0; o >>= 1) key = max(key, (unsigned)__shfl_xor((int)key, o, 32));
            if (r == 0) {
                sh_piv = key ? 255 - (int)(key & 255u) : k;
                sh_pval = (key >> 8) ? 1.0 : 0.0;          // 0: the column is zero (singular)
            }
        }
        __syncthreads();
        const int pr = sh_piv;
        if (tid == 0) {
            pivs[k] = pr;
            if (!(sh_pval > 0.0)) sh_singular = 1;
        }
        if (pr != k) {
            const int p32 = pr & 31, pq = pr >> 5;
            if (r == k32 || r == p32) {
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) {
                    const int j = cc + 32 * jj;
                    const c64 vk = a[kq][jj];
                    c64 vp = a[0][jj];
#pragma unroll
                    for (int t = 1; t < NB; ++t)
                        if (pq == t) vp = a[t][jj];
                    if (j < m) {
                        if (r == k32) row_k[j] = vk;
                        if (r == p32) row_p[j] = vp;
                    }
                }
            }
            __syncthreads();
            if (r == k32 || r == p32) {
#pragma unroll
                for (int jj = 0; jj < NB; ++jj) {
                    const int j = cc + 32 * jj;
                    if (j >= m) continue;
                    const c64 nk = row_p[j], np = row_k[j];
                    if (r == k32) a[kq][jj] = nk;
#pragma unroll
                    for (int t = 0; t < NB; ++t)
                        if (r == p32 && pq == t) a[t][jj] = np;
                }
            }
        }
        if (r == k32) {                                    // publish the pivot row (columns >= k)
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
                const int j = cc + 32 * jj;
                if (j >= k && j < m) ubuf[j] = a[kq][jj];
            }
        }
        __syncthreads();
        const c64 pivot = ubuf[k];
        if (tid == 0) diag[k] = pivot;
        const c64 ip = cinv(pivot);
        if (cc == k32) {                                   // multipliers of column k
#pragma unroll
            for (int ii = 0; ii < NB; ++ii) {
                const int i = r + 32 * ii;
                const c64 l = a[ii][kq] * ip;
                if (i > k && i < m) {
                    a[ii][kq] = l;
                    lbuf[i] = l;
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < NB; ++ii) {
            const int i = r + 32 * ii;
            if (i <= k || i >= m) continue;
            const c64 l = lbuf[i];
#pragma unroll
            for (int jj = 0; jj < NB; ++jj) {
                const int j = cc + 32 * jj;
                if (j > k && j < m) a[ii][jj] = a[ii][jj] - l * ubuf[j];
            }
        }
    }
    if (tid == 0) {                                        // row permutation of the factorisation
        for (int i = 0; i < m; ++i) perm[i] = i;
        for (int k = 0; k < m; ++k) {
            const int q = pivs[k];
            const int t = perm[k];
            perm[k] = perm[q];
            perm[q] = t;
        }
    }
    __syncthreads();
    // pivot growth from the pivots kept in diag (not carried through the
    // elimination, where the two extra live values spilled to scratch)
    double umax = 0.0, umin = 1e308;
    for (int i = tid; i < m; i += blockDim.x) {
        const double pm = cmod(diag[i]);
        umax = fmax(umax, pm);
        umin = fmin(umin, pm);
    }
    umax = block_max(umax, red);
    umin = -block_max(-umin, red);

    // right-hand sides: applied voltages (ADJ: the given ones) and ones, permuted
    const c64* bf = ADJ ? rhs + (size_t)f * p.n : nullptr;
    auto bval = [&](int i) -> c64 { return ADJ ? bf[i] : c64{vapp[colof[i]], 0.0}; };
    for (int i = tid; i < m; i += blockDim.x) {
        y1[i] = bval(perm[i]);
        y2[i] = c64{1.0, 0.0};
    }
    solve_in_registers<NB>(a, m, r, cc, diag, y1, y2, true);
    // c = (1' x1) / (1' x2);  q' = x1 - c x2
    c64 s1{0.0, 0.0}, s2{0.0, 0.0};
    for (int i = tid; i < m; i += blockDim.x) {
        s1 = s1 + y1[i];
        s2 = s2 + y2[i];
    }
    const c64 t1 = block_csum(s1, redc), t2 = block_csum(s2, redc);
    const c64 cg = t1 * cinv(t2);
    for (int i = tid; i < m; i += blockDim.x) {
        xq[i] = y1[i] - cg * y2[i];
        rr[i] = y2[i];                                     // keep St^-1 1 for the corrections
    }
    if (tid == 0) sh_c = cg;
    __syncthreads();

    // infinity norms of the bordered system and of b
    double srow = 0.0;
    for (int i = wave; i < m; i += nwave) {
        double sacc = 0.0;
        for (int j = lane; j < m; j += 64) sacc += cmod(st(i, j));
        for (int o = 32; o > 0; o >>= 1) sacc += __shfl_xor(sacc, o, 64);
        srow = fmax(srow, sacc + 1.0);
    }
    const double snorm = fmax(block_max(srow, red), (double)m);
    double bmax = 0.0;
    if constexpr (ADJ) {
        for (int i = tid; i < m; i += blockDim.x) bmax = fmax(bmax, cmod(bf[i]));
        bmax = block_max(bmax, red);
    } else {
        for (int w = 0; w < p.n_cols; ++w) bmax = fmax(bmax, fabs(vapp[w]));
    }
    const c64 s2_all = t2;

    int iters = 0;
    double berr = 0.0;
    for (;;) {
        // residual of the bordered system: rows i < m into y1, neutrality into redc-sum
        const c64 cur_c = sh_c;
        double rmax = 0.0;
        for (int i = wave; i < m; i += nwave) {
            c64 acc{0.0, 0.0};
            for (int j = lane; j < m; j += 64) acc = acc + st(i, j) * xq[j];
            for (int o = 32; o > 0; o >>= 1) {
                acc.re += __shfl_xor(acc.re, o, 64);
                acc.im += __shfl_xor(acc.im, o, 64);
            }
            const c64 ri = bval(i) - acc - cur_c;
            if (lane == 0) y1[i] = ri;
            rmax = fmax(rmax, cmod(ri));
        }
        c64 qs{0.0, 0.0};
        double xmax = 0.0;
        for (int i = tid; i < m; i += blockDim.x) {
            qs = qs + xq[i];
            xmax = fmax(xmax, cmod(xq[i]));
        }
        const c64 r2 = c64{0.0, 0.0} - block_csum(qs, redc);
        rmax = fmax(block_max(rmax, red), cmod(r2));
        xmax = fmax(block_max(xmax, red), cmod(cur_c));
        const double den = snorm * xmax + bmax;
        berr = den > 0.0 ? rmax / den : 0.0;
        if (berr <= p.ir_tol || iters >= p.ir_max_iter) break;
        // correction: d = St^-1 r1 - dc x2,  dc = (1' St^-1 r1 - r2) / (1' x2)
        for (int i = tid; i < m; i += blockDim.x) y2[i] = y1[perm[i]];
        __syncthreads();
        for (int i = tid; i < m; i += blockDim.x) y1[i] = y2[i];
        solve_in_registers<NB>(a, m, r, cc, diag, y1, y2, false);
        c64 sd{0.0, 0.0};
        for (int i = tid; i < m; i += blockDim.x) sd = sd + y1[i];
        const c64 dc = (block_csum(sd, redc) - r2) * cinv(s2_all);
        for (int i = tid; i < m; i += blockDim.x) xq[i] = xq[i] + y1[i] - dc * rr[i];
        if (tid == 0) sh_c = cur_c + dc;
        __syncthreads();
        ++iters;
    }

    const int n = p.n;
    for (int i = tid; i < m; i += blockDim.x) qw[(size_t)f * n + i] = scale(xq[i], inv_a);
    if (tid == 0) {
        qw[(size_t)f * n + m] = sh_c;
        rep[f].backward_error = berr;
        rep[f].pivot_ratio = umin > 0.0 ? umax / umin : 1e308;
        rep[f].iters = iters;
        rep[f].singular = sh_singular;
    }
}

}  // namespace

hipError_t launch_collocation_solve(const Plan& p, void* ws, hipStream_t s) {
    char* b = static_cast<char*>(ws);
    const double* A = (const double*)(b + p.off_A);
    c64* lu = (c64*)(b + p.off_lu);
    int* piv = (int*)(b + p.off_piv);
    c64* qw = (c64*)(b + p.off_qw);
    SolveReport* rep = (SolveReport*)(b + p.off_rep);
    if (p.n_q <= 64) {
        hipLaunchKernelGGL((k_solve_schur<2, false>), dim3(p.n_freq), dim3(1024), 0, s, p, A, nullptr, qw, rep);
        return hipGetLastError();
    }
    if (p.n_q <= 96) {
        hipLaunchKernelGGL((k_solve_schur<3, false>), dim3(p.n_freq), dim3(1024), 0, s, p, A, nullptr, qw, rep);
        return hipGetLastError();
    }
    if (p.n_q <= 128) {
        hipLaunchKernelGGL((k_solve_schur<4, false>), dim3(p.n_freq), dim3(1024), 0, s, p, A, nullptr, qw, rep);
        return hipGetLastError();
    }
    if (p.n <= 144) {
        hipLaunchKernelGGL((k_solve_reg<16, 9, 5>), dim3(p.n_freq), dim3(512), 0, s, p, A, lu, piv, qw, rep);
        return hipGetLastError();
    }
    const size_t lds = std::max((size_t)kMaxN * kPanel, (size_t)2 * kMaxN) * sizeof(c64);
    hipError_t e = hipFuncSetAttribute((const void*)k_solve_blocked, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_solve_blocked, dim3(p.n_freq), dim3(kBlockedThreads), lds, s, p,
                       (const double*)(b + p.off_A), (c64*)(b + p.off_lu), (int*)(b + p.off_piv),
                       (c64*)(b + p.off_qw), (SolveReport*)(b + p.off_rep));
    return hipGetLastError();
}

// Transposed systems of the adjoint (Schur form only: n_q <= 128).
hipError_t launch_adjoint_solve(const Plan& p, const void* ws, const void* rhs, void* lam, void* rep,
                                hipStream_t s) {
    const double* A = (const double*)(static_cast<const char*>(ws) + p.off_A);
    const c64* b = static_cast<const c64*>(rhs);
    c64* x = static_cast<c64*>(lam);
    SolveReport* r = static_cast<SolveReport*>(rep);
    if (p.n_q <= 64)
        hipLaunchKernelGGL((k_solve_schur<2, true>), dim3(p.n_freq), dim3(1024), 0, s, p, A, b, x, r);
    else if (p.n_q <= 96)
        hipLaunchKernelGGL((k_solve_schur<3, true>), dim3(p.n_freq), dim3(1024), 0, s, p, A, b, x, r);
    else if (p.n_q <= 128)
        hipLaunchKernelGGL((k_solve_schur<4, true>), dim3(p.n_freq), dim3(1024), 0, s, p, A, b, x, r);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace wt
