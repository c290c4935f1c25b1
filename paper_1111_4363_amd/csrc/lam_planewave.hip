// The plane-wave relaxation experiment in the Legendre finite-element basis
// (Sec. "Implementation with Legendre Polynomials", Sec. "Convergence"):
// host construction of the element operators and of the linear maps of one
// relaxation, and the batched kernel that applies them to a grid of trial
// plane waves exp(i(k x + w t)).
//
// Per element [-1, 1] x [-1, 1] (dimensionless space y and time), basis
// P_i(y) P_n(t), i < n_x, n < n_t, coefficient index (i, n) -> i n_t + n,
// elements stacked.  Least-action operator of one element,
// Eq. (leastaction_dimensionless), row = test (j, m), column = trial (i, n):
//   A = i O (x) Q^T - 2 kappa T^T (x) U - nu O (x) U   (entries below),
// with O_ij = 2 delta_ij / (2i + 1), U likewise, Q_nm = 2 for n > m, n - m
// odd, and T_ij = (j(j+1) - i(i+1)) / 2 for i > j, i - j even: the entry of
// trial i in test row j (the closed form the paper prints; its printed
// integral exchanges i and j).
//
// One relaxation maps the trial's residual r = -A C to a correction
// delta = M r that vanishes at the initial time and on the boundary of the
// relaxation volume and is continuous inside it, and makes the new residual
// orthogonal to every such correction (Eq. (leastaction_correction) with
// Eqs. (ic_correction), (bc1_correction), (bc2_correction)): with N an
// orthonormal basis of the admissible corrections, M = N (N^T A N)^{-1} N^T.
// Modes: one element; two elements simultaneously; two elements by intergrid
// transfer (Eqs. (residual_rough), (correction_fine): parent problem
// P A I with P the overlap-weighted transpose of the interpolation I, so
// P I = identity, then each element with its interface fixed).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "lam_internal.h"

namespace {

using cd = std::complex<double>;
using Mat = std::vector<cd>;      // row-major n x n (or r x c with the sizes alongside)
using RMat = std::vector<double>;

constexpr int kQ = 64;            // quadrature nodes for the trial's overlaps
constexpr int kPT = 32;           // trial points per workgroup
constexpr int kPWThreads = 256;   // 8 row groups x 32 points

double legendre(int n, double y) {
    double p0 = 1.0, p1 = y;
    if (n == 0) return 1.0;
    for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * y * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
    }
    return p1;
}

// Gauss-Legendre nodes and weights (Newton on P_N from the usual cosine start).
void gauss_nodes(int N, double* x, double* w) {
    for (int i = 0; i < N; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (N + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            const double p = legendre(N, z), q = legendre(N - 1, z);
            dp = N * (z * p - q) / (z * z - 1.0);
            const double dz = p / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        const double p = legendre(N, z), q = legendre(N - 1, z);
        dp = N * (z * p - q) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

RMat matmul(const RMat& a, const RMat& b, int r, int k, int c) {
    RMat o((size_t)r * c, 0.0);
    for (int i = 0; i < r; ++i)
        for (int l = 0; l < k; ++l)
            for (int j = 0; j < c; ++j) o[(size_t)i * c + j] += a[(size_t)i * k + l] * b[(size_t)l * c + j];
    return o;
}

template <typename T>
std::vector<T> transpose(const std::vector<T>& a, int r, int c) {
    std::vector<T> o((size_t)r * c);
    for (int i = 0; i < r; ++i)
        for (int j = 0; j < c; ++j) o[(size_t)j * r + i] = a[(size_t)i * c + j];
    return o;
}

// In-place inverse of an n x n matrix (Gauss-Jordan, partial pivoting).
template <typename T>
bool invert(std::vector<T>& A, int n) {
    std::vector<int> piv(n);
    for (int col = 0; col < n; ++col) {
        int p = col;
        for (int r = col + 1; r < n; ++r)
            if (std::abs(A[(size_t)r * n + col]) > std::abs(A[(size_t)p * n + col])) p = r;
        piv[col] = p;
        if (std::abs(A[(size_t)p * n + col]) == 0.0) return false;
        if (p != col)
            for (int k = 0; k < n; ++k) std::swap(A[(size_t)col * n + k], A[(size_t)p * n + k]);
        const T inv = T(1.0) / A[(size_t)col * n + col];
        A[(size_t)col * n + col] = T(1.0);
        for (int k = 0; k < n; ++k) A[(size_t)col * n + k] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const T f = A[(size_t)r * n + col];
            A[(size_t)r * n + col] = T(0.0);
            for (int k = 0; k < n; ++k) A[(size_t)r * n + k] -= f * A[(size_t)col * n + k];
        }
    }
    for (int col = n - 1; col >= 0; --col)
        if (piv[col] != col)
            for (int r = 0; r < n; ++r) std::swap(A[(size_t)r * n + col], A[(size_t)r * n + piv[col]]);
    return true;
}

// Least-action operator of one element (see the file comment).
Mat element_operator(int nx, int nt, double kappa, double nu) {
    const int n = nx * nt;
    Mat A((size_t)n * n, 0.0);
    auto O = [](int i) { return 2.0 / (2.0 * i + 1.0); };
    for (int j = 0; j < nx; ++j)
        for (int m = 0; m < nt; ++m)
            for (int i = 0; i < nx; ++i)
                for (int q = 0; q < nt; ++q) {
                    cd v = 0.0;
                    if (i == j && q > m && ((q - m) & 1)) v += cd(0.0, O(i) * 2.0);       // i O_ij Q_qm
                    if (q == m && i > j && !((i - j) & 1))
                        v -= 2.0 * kappa * 0.5 * (j * (j + 1.0) - i * (i + 1.0)) * O(q);  // -2 kappa T_ij U_qm
                    if (i == j && q == m) v -= nu * O(i) * O(q);                          // -nu O_ij U_qm
                    A[(size_t)(j * nt + m) * n + i * nt + q] = v;
                }
    return A;
}

// Rows of the constraints on a correction over ne elements: zero at the
// initial time in each element, at the left and right ends, and at the
// interface either continuous (interface_fixed = false) or zero on both sides.
// The rows repeat each other at the corners; the null space below copes with
// that.
RMat constraint_rows(int nx, int nt, int ne, bool ends, bool interface_fixed, int* rows) {
    const int nel = nx * nt, n = ne * nel;
    RMat B;
    auto add = [&](const std::vector<double>& r) { B.insert(B.end(), r.begin(), r.end()); };
    auto sgn = [](int k) { return (k & 1) ? -1.0 : 1.0; };
    for (int e = 0; e < ne; ++e)
        for (int i = 0; i < nx; ++i) {
            std::vector<double> r(n, 0.0);
            for (int q = 0; q < nt; ++q) r[e * nel + i * nt + q] = sgn(q);
            add(r);
        }
    for (int q = 0; q < nt; ++q) {
        if (ends) {
            std::vector<double> l(n, 0.0), r(n, 0.0);
            for (int i = 0; i < nx; ++i) {
                l[i * nt + q] = sgn(i);
                r[(ne - 1) * nel + i * nt + q] = 1.0;
            }
            add(l);
            add(r);
        }
        if (ne == 2) {
            if (!interface_fixed) {
                std::vector<double> r(n, 0.0);
                for (int i = 0; i < nx; ++i) {
                    r[i * nt + q] = 1.0;
                    r[nel + i * nt + q] = -sgn(i);
                }
                add(r);
            } else {
                std::vector<double> l(n, 0.0), r(n, 0.0);
                for (int i = 0; i < nx; ++i) {
                    l[i * nt + q] = 1.0;
                    r[nel + i * nt + q] = sgn(i);
                }
                add(l);
                add(r);
            }
        }
    }
    *rows = (int)(B.size() / n);
    return B;
}

// Orthonormal basis (columns of an n x d matrix) of {x : B x = 0}: modified
// Gram-Schmidt (twice) of the rows of B, then of the unit vectors against them.
RMat null_space(const RMat& B, int m, int n, int* d) {
    std::vector<std::vector<double>> basis;
    auto reduce = [&](std::vector<double>& v) {
        for (int pass = 0; pass < 2; ++pass)
            for (const auto& q : basis) {
                double dot = 0.0;
                for (int k = 0; k < n; ++k) dot += q[k] * v[k];
                for (int k = 0; k < n; ++k) v[k] -= dot * q[k];
            }
        double nv = 0.0;
        for (double x : v) nv += x * x;
        return std::sqrt(nv);
    };
    for (int r = 0; r < m; ++r) {
        std::vector<double> v(B.begin() + (size_t)r * n, B.begin() + (size_t)(r + 1) * n);
        double n0 = 0.0;
        for (double x : v) n0 += x * x;
        const double nr = reduce(v);
        if (nr > 1e-10 * std::sqrt(n0)) {
            for (double& x : v) x /= nr;
            basis.push_back(v);
        }
    }
    const size_t rank = basis.size();
    for (int j = 0; j < n && (int)basis.size() < n; ++j) {
        std::vector<double> v(n, 0.0);
        v[j] = 1.0;
        const double nr = reduce(v);
        if (nr > 1e-8) {
            for (double& x : v) x /= nr;
            basis.push_back(v);
        }
    }
    *d = (int)(basis.size() - rank);
    RMat N((size_t)n * *d);
    for (int c = 0; c < *d; ++c)
        for (int k = 0; k < n; ++k) N[(size_t)k * *d + c] = basis[rank + c][k];
    return N;
}

// M = N (N^T A N)^{-1} N^T for the constraints B (m rows).
bool relax_operator(const Mat& A, int n, const RMat& B, int m, Mat& M) {
    int d = 0;
    const RMat N = null_space(B, m, n, &d);
    M.assign((size_t)n * n, 0.0);
    if (d == 0) return true;
    Mat AN((size_t)n * d, 0.0), R((size_t)d * d, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const cd a = A[(size_t)i * n + k];
            if (a == 0.0) continue;
            for (int c = 0; c < d; ++c) AN[(size_t)i * d + c] += a * N[(size_t)k * d + c];
        }
    for (int r = 0; r < d; ++r)
        for (int i = 0; i < n; ++i) {
            const double q = N[(size_t)i * d + r];
            if (q == 0.0) continue;
            for (int c = 0; c < d; ++c) R[(size_t)r * d + c] += q * AN[(size_t)i * d + c];
        }
    if (!invert(R, d)) return false;
    Mat NR((size_t)n * d, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < d; ++k) {
            const double q = N[(size_t)i * d + k];
            if (q == 0.0) continue;
            for (int c = 0; c < d; ++c) NR[(size_t)i * d + c] += q * R[(size_t)k * d + c];
        }
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < d; ++c) {
            const cd v = NR[(size_t)i * d + c];
            for (int j = 0; j < n; ++j) M[(size_t)i * n + j] += v * N[(size_t)j * d + c];
        }
    return true;
}

Mat cmatmul(const Mat& a, const Mat& b, int r, int k, int c) {
    Mat o((size_t)r * c, 0.0);
    for (int i = 0; i < r; ++i)
        for (int l = 0; l < k; ++l) {
            const cd v = a[(size_t)i * k + l];
            if (v == 0.0) continue;
            for (int j = 0; j < c; ++j) o[(size_t)i * c + j] += v * b[(size_t)l * c + j];
        }
    return o;
}

Mat to_complex(const RMat& a) { return Mat(a.begin(), a.end()); }

// Interpolation parent -> child (child j, parent i: the paper's I_ij / O_jj) for
// the left (shift -1) or right (shift +1) child, and the projections P = G^{-1} I^T O.
void transfers(int n, RMat& IL, RMat& IR, RMat& PL, RMat& PR) {
    double x[kQ], w[kQ];
    gauss_nodes(kQ, x, w);
    RMat O((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) O[(size_t)i * n + i] = 2.0 / (2.0 * i + 1.0);
    for (int side = 0; side < 2; ++side) {
        const double shift = side == 0 ? -1.0 : 1.0;
        RMat I((size_t)n * n, 0.0);
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double acc = 0.0;
                for (int q = 0; q < kQ; ++q) acc += w[q] * legendre(i, 0.5 * (x[q] + shift)) * legendre(j, x[q]);
                I[(size_t)j * n + i] = acc / O[(size_t)j * n + j];
            }
        (side == 0 ? IL : IR) = I;
    }
    RMat G = matmul(transpose(IL, n, n), matmul(O, IL, n, n, n), n, n, n);
    const RMat G2 = matmul(transpose(IR, n, n), matmul(O, IR, n, n, n), n, n, n);
    for (size_t k = 0; k < G.size(); ++k) G[k] += G2[k];
    invert(G, n);
    PL = matmul(G, matmul(transpose(IL, n, n), O, n, n, n), n, n, n);
    PR = matmul(G, matmul(transpose(IR, n, n), O, n, n, n), n, n, n);
}

// The space transfer with the time identity, in the (i, n) layout: [rows_s * nt][cols_s * nt].
RMat kron_time(const RMat& S, int rs, int cs, int nt) {
    RMat o((size_t)rs * nt * cs * nt, 0.0);
    for (int i = 0; i < rs; ++i)
        for (int j = 0; j < cs; ++j)
            for (int q = 0; q < nt; ++q) o[(size_t)(i * nt + q) * (cs * nt) + j * nt + q] = S[(size_t)i * cs + j];
    return o;
}

}  // namespace

namespace lam {

// Everything the kernel reads, in one device buffer.
struct PWTables {
    int n, nx, nt, ne, nk, nw;
    const double2* A;      // n x n
    const double2* M;      // n x n
    const double2* R;      // n x n: I - A M
    const double* Pi;      // n x n continuity projection (two elements), or null
    const double* G;       // n: diagonal of O (x) U per element
    const double* Px;      // [8][kQ] P_i(y_q) w_q  (space)
    const double* Pt;      // [8][kQ] P_n(y_q) w_q  (time)
    const double* yq;      // [kQ] nodes
    const double* k;       // nk
    const double* w;       // nw
};

namespace {

__device__ __forceinline__ double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 add2_(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// One workgroup: 32 trial points (flattened (iw, ik)), 8 row groups of 32 threads.
__global__ __launch_bounds__(kPWThreads) void k_plane_wave(PWTables t, double* __restrict__ rratio,
                                                           double* __restrict__ aratio) {
    __shared__ double2 Cs[LAM_PW_MAX_UNKNOWNS * kPT];   // trial, then relaxed coefficients [row][point]
    __shared__ double2 Rs[LAM_PW_MAX_UNKNOWNS * kPT];   // residual
    __shared__ double2 ab[2 * 8 * kPT];                  // space / time overlaps [i][point]
    __shared__ double red[4 * 8 * kPT];
    const int tid = threadIdx.x, p = tid & (kPT - 1), g = tid >> 5;
    const int n = t.n, nt = t.nt, nx = t.nx;
    const long total = (long)t.nk * t.nw;
    const long pid = (long)blockIdx.x * kPT + p;
    const bool live = pid < total;
    const long pc = live ? pid : 0;
    const int iw = (int)(pc / t.nk), ik = (int)(pc - (long)iw * t.nk);
    const double kk = t.k[ik], ww = t.w[iw];
    // 1. overlaps int P_g(y) exp(i s y) dy of the point's wave numbers (s = k, or k/2 on
    //    the two elements' own coordinates) and int P_g(t) exp(i w t) dt
    const double ks = t.ne == 2 ? 0.5 * kk : kk;
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
    for (int q = 0; q < kQ; ++q) {
        double sn, cs;
        sincos(ks * t.yq[q], &sn, &cs);
        a.x += t.Px[g * kQ + q] * cs;
        a.y += t.Px[g * kQ + q] * sn;
        sincos(ww * t.yq[q], &sn, &cs);
        b.x += t.Pt[g * kQ + q] * cs;
        b.y += t.Pt[g * kQ + q] * sn;
    }
    ab[g * kPT + p] = a;
    ab[(8 + g) * kPT + p] = b;
    __syncthreads();
    // 2. element coefficients (L2 projection: overlaps over O (x) U), element phases
    //    exp(-+ i k/2) for two elements; rows g, g + 8, ...
    for (int r = g; r < n; r += 8) {
        const int e = r / (nx * nt), ri = r - e * nx * nt, i = ri / nt, q = ri - i * nt;
        double2 v = cmul2(ab[i * kPT + p], ab[(8 + q) * kPT + p]);
        if (t.ne == 2) {
            double sn, cs;
            sincos((e == 0 ? -0.5 : 0.5) * kk, &sn, &cs);
            v = cmul2(v, make_double2(cs, sn));
        }
        Rs[r * kPT + p] = make_double2(v.x / t.G[r], v.y / t.G[r]);
    }
    __syncthreads();
    // continuity across the interface (two elements): C = Pi C_local
    for (int r = g; r < n; r += 8) {
        double2 v;
        if (t.Pi) {
            v = make_double2(0.0, 0.0);
            for (int c = 0; c < n; ++c) {
                const double s = t.Pi[r * n + c];
                const double2 x = Rs[c * kPT + p];
                v.x += s * x.x;
                v.y += s * x.y;
            }
        } else {
            v = Rs[r * kPT + p];
        }
        Cs[r * kPT + p] = v;
    }
    __syncthreads();
    // 3. r = -A C, and the action and residual norm of the trial
    double n0 = 0.0, s0r = 0.0, s0i = 0.0;
    for (int r = g; r < n; r += 8) {
        double2 v = make_double2(0.0, 0.0);
        for (int c = 0; c < n; ++c) v = add2_(v, cmul2(t.A[r * n + c], Cs[c * kPT + p]));
        v = make_double2(-v.x, -v.y);
        Rs[r * kPT + p] = v;
        n0 += t.G[r] * (v.x * v.x + v.y * v.y);
        const double2 cr = Cs[r * kPT + p];   // S = C^H A C = -C^H r
        s0r -= cr.x * v.x + cr.y * v.y;
        s0i -= cr.x * v.y - cr.y * v.x;
    }
    __syncthreads();
    // 4. delta = M r, r' = R r; C' = C + delta
    double n1 = 0.0, s1r = 0.0, s1i = 0.0;
    constexpr int kRowSlots = (LAM_PW_MAX_UNKNOWNS + 7) / 8;
#pragma unroll
    for (int slot = 0; slot < kRowSlots; ++slot) {
        const int r = g + 8 * slot;
        if (r >= n) break;
        double2 dv = make_double2(0.0, 0.0), rv = make_double2(0.0, 0.0);
        for (int c = 0; c < n; ++c) {
            const double2 x = Rs[c * kPT + p];
            dv = add2_(dv, cmul2(t.M[r * n + c], x));
            rv = add2_(rv, cmul2(t.R[r * n + c], x));
        }
        const double2 cr = Cs[r * kPT + p];
        const double2 c2 = make_double2(cr.x + dv.x, cr.y + dv.y);
        n1 += t.G[r] * (rv.x * rv.x + rv.y * rv.y);
        s1r -= c2.x * rv.x + c2.y * rv.y;     // S' = -C'^H r'
        s1i -= c2.x * rv.y - c2.y * rv.x;
    }
    // 5. sums over the 8 row groups of each point, in a fixed order
    red[(0 * 8 + g) * kPT + p] = n0;
    red[(1 * 8 + g) * kPT + p] = n1;
    red[(2 * 8 + g) * kPT + p] = s0r;
    red[(3 * 8 + g) * kPT + p] = s0i;
    __syncthreads();
    double N0 = 0.0, N1 = 0.0, S0r = 0.0, S0i = 0.0;
    if (g == 0)
        for (int k = 0; k < 8; ++k) {
            N0 += red[(0 * 8 + k) * kPT + p];
            N1 += red[(1 * 8 + k) * kPT + p];
            S0r += red[(2 * 8 + k) * kPT + p];
            S0i += red[(3 * 8 + k) * kPT + p];
        }
    __syncthreads();
    red[(0 * 8 + g) * kPT + p] = s1r;
    red[(1 * 8 + g) * kPT + p] = s1i;
    __syncthreads();
    if (g == 0 && live) {
        double S1r = 0.0, S1i = 0.0;
        for (int k = 0; k < 8; ++k) {
            S1r += red[(0 * 8 + k) * kPT + p];
            S1i += red[(1 * 8 + k) * kPT + p];
        }
        rratio[pid] = sqrt(N1 / N0);
        aratio[pid] = sqrt(S1r * S1r + S1i * S1i) / sqrt(S0r * S0r + S0i * S0i);
    }
}

}  // namespace
}  // namespace lam

namespace {

// The linear maps of one relaxation of the given mode (A: operator over its
// elements, M: residual -> correction), and the continuity projection of the
// two-element trial.  false if a reduced system is singular.
bool mode_maps(const lam_pw_regime& rg, int ne, Mat& A, Mat& M, RMat& Pi) {
    const int nx = rg.n_x, nt = rg.n_t, nel = nx * nt, n = ne * nel;
    const Mat A1 = element_operator(nx, nt, rg.kappa, rg.nu);
    A.assign((size_t)n * n, 0.0);
    for (int e = 0; e < ne; ++e)
        for (int i = 0; i < nel; ++i)
            for (int j = 0; j < nel; ++j) A[(size_t)(e * nel + i) * n + e * nel + j] = A1[(size_t)i * nel + j];
    int m = 0;
    if (rg.mode == LAM_PW_ONE || rg.mode == LAM_PW_SIMULTANEOUS) {
        const RMat B = constraint_rows(nx, nt, ne, true, false, &m);
        if (!relax_operator(A, n, B, m, M)) return false;
    } else {
        RMat IL, IR, PL, PR;
        transfers(nx, IL, IR, PL, PR);
        // Pr: parent <- children (nel x n), Ip: children <- parent (n x nel)
        const RMat pl = kron_time(PL, nx, nx, nt), pr = kron_time(PR, nx, nx, nt);
        const RMat il = kron_time(IL, nx, nx, nt), ir = kron_time(IR, nx, nx, nt);
        RMat Pr((size_t)nel * n), Ip((size_t)n * nel);
        for (int r = 0; r < nel; ++r)
            for (int c = 0; c < nel; ++c) {
                Pr[(size_t)r * n + c] = pl[(size_t)r * nel + c];
                Pr[(size_t)r * n + nel + c] = pr[(size_t)r * nel + c];
                Ip[(size_t)r * nel + c] = il[(size_t)r * nel + c];
                Ip[(size_t)(nel + r) * nel + c] = ir[(size_t)r * nel + c];
            }
        const Mat Prc = to_complex(Pr), Ipc = to_complex(Ip);
        const Mat Ac = cmatmul(Prc, cmatmul(A, Ipc, n, n, nel), nel, n, nel);
        Mat Mc, Mf;
        int mc = 0, mf = 0;
        const RMat Bc = constraint_rows(nx, nt, 1, true, false, &mc);
        const RMat Bf = constraint_rows(nx, nt, 2, true, true, &mf);
        if (!relax_operator(Ac, nel, Bc, mc, Mc)) return false;
        if (!relax_operator(A, n, Bf, mf, Mf)) return false;
        // M = Mco + Mf (I - A Mco) with Mco = Ip Mc Pr
        const Mat Mco = cmatmul(Ipc, cmatmul(Mc, Prc, nel, nel, n), n, nel, n);
        Mat IAM = cmatmul(A, Mco, n, n, n);
        for (auto& v : IAM) v = -v;
        for (int i = 0; i < n; ++i) IAM[(size_t)i * n + i] += 1.0;
        M = cmatmul(Mf, IAM, n, n, n);
        for (size_t k = 0; k < M.size(); ++k) M[k] += Mco[k];
    }
    Pi.clear();
    if (ne == 2) {
        // C = C_local - G^{-1} Bc^T (Bc G^{-1} Bc^T)^{-1} Bc C_local, Bc the continuity rows
        std::vector<double> G(n);
        for (int e = 0; e < ne; ++e)
            for (int i = 0; i < nx; ++i)
                for (int q = 0; q < nt; ++q)
                    G[e * nel + i * nt + q] = (2.0 / (2.0 * i + 1.0)) * (2.0 / (2.0 * q + 1.0));
        RMat Bc((size_t)nt * n, 0.0);
        for (int q = 0; q < nt; ++q)
            for (int i = 0; i < nx; ++i) {
                Bc[(size_t)q * n + i * nt + q] = 1.0;
                Bc[(size_t)q * n + nel + i * nt + q] = -((i & 1) ? -1.0 : 1.0);
            }
        RMat S((size_t)nt * nt, 0.0);
        for (int a = 0; a < nt; ++a)
            for (int b2 = 0; b2 < nt; ++b2)
                for (int c = 0; c < n; ++c) S[(size_t)a * nt + b2] += Bc[(size_t)a * n + c] * Bc[(size_t)b2 * n + c] / G[c];
        if (!invert(S, nt)) return false;
        Pi.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i) Pi[(size_t)i * n + i] = 1.0;
        // Pi -= G^{-1} Bc^T S^{-1} Bc
        for (int i = 0; i < n; ++i)
            for (int a = 0; a < nt; ++a) {
                const double left = Bc[(size_t)a * n + i] / G[i];
                if (left == 0.0) continue;
                for (int b2 = 0; b2 < nt; ++b2) {
                    const double f = left * S[(size_t)a * nt + b2];
                    for (int j = 0; j < n; ++j) Pi[(size_t)i * n + j] -= f * Bc[(size_t)b2 * n + j];
                }
            }
    }
    return true;
}

}  // namespace

extern "C" int lam_plane_wave_map(const lam_pw_regime* regime, int nk, const double* k, int nw, const double* w,
                                  double* resid_ratio, double* action_ratio, void* hip_stream) {
    if (!regime || !k || !w || !resid_ratio || !action_ratio || nk < 1 || nw < 1) return LAM_EINVAL;
    const lam_pw_regime& rg = *regime;
    if (rg.n_x < 1 || rg.n_x > 8 || rg.n_t < 1 || rg.n_t > 8) return LAM_EINVAL;
    if (rg.mode != LAM_PW_ONE && rg.mode != LAM_PW_SIMULTANEOUS && rg.mode != LAM_PW_INTERGRID) return LAM_EINVAL;
    if (!std::isfinite(rg.kappa) || !std::isfinite(rg.nu)) return LAM_EINVAL;
    const int ne = rg.mode == LAM_PW_ONE ? 1 : 2;
    const int n = ne * rg.n_x * rg.n_t;
    if (n > LAM_PW_MAX_UNKNOWNS) return LAM_EINVAL;
    if ((long)nk * nw > (1L << 30)) return LAM_EINVAL;
    Mat A, M;
    RMat Pi;
    if (!mode_maps(rg, ne, A, M, Pi)) return LAM_EINVAL;
    Mat R = cmatmul(A, M, n, n, n);
    for (auto& v : R) v = -v;
    for (int i = 0; i < n; ++i) R[(size_t)i * n + i] += 1.0;
    // quadrature tables
    double yq[kQ], wq[kQ];
    gauss_nodes(kQ, yq, wq);
    // one host buffer of doubles: A, M, R (complex), Pi, G, Px, Pt, yq, k, w
    const size_t nA = 2 * (size_t)n * n, nPi = Pi.empty() ? 0 : (size_t)n * n;
    std::vector<double> h;
    h.reserve(3 * nA + nPi + n + 2 * 8 * kQ + kQ + nk + nw);
    size_t off_A = h.size();
    for (const Mat* X : {&A, &M, &R})
        for (const cd& v : *X) {
            h.push_back(v.real());
            h.push_back(v.imag());
        }
    const size_t off_Pi = h.size();
    h.insert(h.end(), Pi.begin(), Pi.end());
    const size_t off_G = h.size();
    for (int e = 0; e < ne; ++e)
        for (int i = 0; i < rg.n_x; ++i)
            for (int q = 0; q < rg.n_t; ++q) h.push_back((2.0 / (2.0 * i + 1.0)) * (2.0 / (2.0 * q + 1.0)));
    const size_t off_Px = h.size();
    for (int i = 0; i < 8; ++i)
        for (int q = 0; q < kQ; ++q) h.push_back(i < rg.n_x ? legendre(i, yq[q]) * wq[q] : 0.0);
    const size_t off_Pt = h.size();
    for (int i = 0; i < 8; ++i)
        for (int q = 0; q < kQ; ++q) h.push_back(i < rg.n_t ? legendre(i, yq[q]) * wq[q] : 0.0);
    const size_t off_y = h.size();
    h.insert(h.end(), yq, yq + kQ);
    const size_t off_k = h.size();
    h.insert(h.end(), k, k + nk);
    const size_t off_w = h.size();
    h.insert(h.end(), w, w + nw);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    double* d = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&d), sizeof(double) * h.size()) != hipSuccess) {
        (void)hipGetLastError();
        return LAM_ENOMEM;
    }
    int rc = LAM_OK;
    do {
        if (hipMemcpyAsync(d, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
            rc = LAM_EHIP;
            break;
        }
        lam::PWTables t{};
        t.n = n;
        t.nx = rg.n_x;
        t.nt = rg.n_t;
        t.ne = ne;
        t.nk = nk;
        t.nw = nw;
        t.A = reinterpret_cast<const double2*>(d + off_A);
        t.M = t.A + (size_t)n * n;
        t.R = t.M + (size_t)n * n;
        t.Pi = nPi ? d + off_Pi : nullptr;
        t.G = d + off_G;
        t.Px = d + off_Px;
        t.Pt = d + off_Pt;
        t.yq = d + off_y;
        t.k = d + off_k;
        t.w = d + off_w;
        const long total = (long)nk * nw;
        const int blocks = (int)((total + kPT - 1) / kPT);
        hipLaunchKernelGGL(lam::k_plane_wave, dim3(blocks), dim3(kPWThreads), 0, st, t, resid_ratio, action_ratio);
        if (hipGetLastError() != hipSuccess) {
            rc = LAM_EHIP;
            break;
        }
        // the tables are freed below: wait for the kernel
        if (hipStreamSynchronize(st) != hipSuccess) rc = LAM_EHIP;
    } while (false);
    if (rc != LAM_OK) (void)hipStreamSynchronize(st);
    (void)hipFree(d);
    return rc;
}
