// Host side of liblam: context, level hierarchy, factorisation, V-cycle,
// step solve and adjoint step.  Every numerical step runs in the kernels of
// lam_kernels.hip; this file only sizes, orders and launches them.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "lam_internal.h"

using namespace lam;

namespace {

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return LAM_EHIP;      \
    } while (0)

#define LAMCHK(x)                                   \
    do {                                            \
        int r_ = (x);                               \
        if (r_ != LAM_OK) return r_;                \
    } while (0)

struct Level {
    LevelGeom g{};
    int nblocks = 0;
    int ncol[2] = {0, 0};
    int* d_blocks[2] = {nullptr, nullptr};
    double* d_v0 = nullptr;
    double2* d_c = nullptr;     // state x = (c, lambda)
    double2* d_lam = nullptr;
    double2* d_bc = nullptr;    // right-hand side (coarse levels)
    double2* d_bs = nullptr;
    double* d_V = nullptr;      // block eigenvectors (FP64)
    double* d_e = nullptr;      // block eigenvalues
    float* d_Vf = nullptr;      // FP32 copy (mixed path)
    double2* d_Minv = nullptr;  // per-mode time-system inverses
    float2* d_Minvf = nullptr;
    unsigned char* d_passes = nullptr;  // per block: inner passes of its last solve
    int nslab = 0;              // blocks along the field axis
    std::vector<double> zslab;  // centre coordinate of each slab along the field axis
    size_t tf_off = 0;          // first record of this level in the slab factor tables
    bool fp32 = false;
};

constexpr int kGL = 48;   // Gauss-Legendre nodes of the field quadrature

// Gauss-Legendre nodes and weights on [-1, 1] by Newton iteration on P_N.
void gauss_legendre(int N, double* x, double* w) {
    for (int i = 0; i < N; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (N + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= N; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = N * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= N; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = N * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// The field quadrature's nodes, computed once.
struct GaussNodes {
    double x[kGL], w[kGL];
    GaussNodes() { gauss_legendre(kGL, x, w); }
};
const GaussNodes& gauss_nodes() {
    static const GaussNodes g;
    return g;
}

// ---------------------------------------------------------------------------
// Small dense complex linear algebra for the time factors of the per-mode
// block systems (n <= 8): fixed-size arrays, no allocation.
// ---------------------------------------------------------------------------
using cd = std::complex<double>;
constexpr int kTN = kMaxNT;   // leading dimension of the small matrices

// In-place inverse of an n x n complex matrix (stride kTN; Gauss-Jordan with
// partial pivoting).  Returns false for an exactly singular pivot.
bool invert_small(int n, cd (*A)[kTN]) {
    int piv[kTN];
    for (int col = 0; col < n; ++col) {
        int p = col;
        for (int r = col + 1; r < n; ++r)
            if (std::abs(A[r][col]) > std::abs(A[p][col])) p = r;
        piv[col] = p;
        if (std::abs(A[p][col]) == 0.0) return false;
        if (p != col)
            for (int k = 0; k < n; ++k) std::swap(A[col][k], A[p][k]);
        const cd inv = 1.0 / A[col][col];
        A[col][col] = 1.0;
        for (int k = 0; k < n; ++k) A[col][k] *= inv;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const cd f = A[r][col];
            A[r][col] = 0.0;
            for (int k = 0; k < n; ++k) A[r][k] -= f * A[col][k];
        }
    }
    for (int col = n - 1; col >= 0; --col)
        if (piv[col] != col)
            for (int r = 0; r < n; ++r) std::swap(A[r][col], A[r][piv[col]]);
    return true;
}

// Complex Schur form H = Z T Z^H of the m x m matrix H (overwritten by the
// upper triangular T; Z unitary): Householder reduction to Hessenberg form,
// then single-shift QR sweeps of Givens rotations with Wilkinson shifts and
// deflation of negligible subdiagonal entries.  false if it does not converge.
bool schur_small(int m, cd (*H)[kTN], cd (*Z)[kTN]) {
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) Z[i][j] = (i == j) ? 1.0 : 0.0;
    double nrm = 0.0;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) nrm += std::norm(H[i][j]);
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return true;
    // Hessenberg: reflector I - 2 v v^H / (v^H v) zeroes H[k+2.., k]
    for (int k = 0; k + 2 < m; ++k) {
        cd v[kTN];
        double xn = 0.0;
        for (int i = k + 1; i < m; ++i) xn += std::norm(H[i][k]);
        xn = std::sqrt(xn);
        if (xn == 0.0) continue;
        const cd x0 = H[k + 1][k];
        const cd ph = std::abs(x0) > 0.0 ? x0 / std::abs(x0) : cd(1.0);
        double vn = 0.0;
        for (int i = k + 1; i < m; ++i) {
            v[i] = H[i][k] + (i == k + 1 ? ph * xn : cd(0.0));
            vn += std::norm(v[i]);
        }
        if (vn == 0.0) continue;
        for (int j = 0; j < m; ++j) {  // H <- P H
            cd d = 0.0;
            for (int i = k + 1; i < m; ++i) d += std::conj(v[i]) * H[i][j];
            d *= 2.0 / vn;
            for (int i = k + 1; i < m; ++i) H[i][j] -= v[i] * d;
        }
        for (int i = 0; i < m; ++i) {  // H <- H P, Z <- Z P
            cd d = 0.0, e = 0.0;
            for (int j = k + 1; j < m; ++j) {
                d += H[i][j] * v[j];
                e += Z[i][j] * v[j];
            }
            d *= 2.0 / vn;
            e *= 2.0 / vn;
            for (int j = k + 1; j < m; ++j) {
                H[i][j] -= d * std::conj(v[j]);
                Z[i][j] -= e * std::conj(v[j]);
            }
        }
        for (int i = k + 2; i < m; ++i) H[i][k] = 0.0;
    }
    const double eps = 1e-16;
    int hi = m - 1, iter = 0;
    while (hi > 0) {
        // the active window [lo, hi] ends at the first negligible subdiagonal entry
        int lo = hi;
        while (lo > 0) {
            const double s = std::abs(H[lo][lo]) + std::abs(H[lo - 1][lo - 1]);
            if (std::abs(H[lo][lo - 1]) <= eps * (s > 0.0 ? s : nrm)) {
                H[lo][lo - 1] = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (++iter > 60) return false;
        // Wilkinson shift from the trailing 2 x 2 block (an exceptional one now and then)
        const cd a = H[hi - 1][hi - 1], b = H[hi - 1][hi], c = H[hi][hi - 1], d = H[hi][hi];
        const cd tr = 0.5 * (a + d);
        const cd disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
        cd mu = (std::abs(tr + disc - d) < std::abs(tr - disc - d)) ? tr + disc : tr - disc;
        if (iter % 10 == 0) mu += 0.75 * std::abs(c);
        for (int i = lo; i <= hi; ++i) H[i][i] -= mu;
        double cs[kTN];
        cd sn[kTN];
        for (int k = lo; k < hi; ++k) {  // H - mu I = Q R: rotations from the left
            const cd x = H[k][k], y = H[k + 1][k];
            const double r = std::sqrt(std::norm(x) + std::norm(y));
            double cc;
            cd ss;
            if (r == 0.0) {
                cc = 1.0;
                ss = 0.0;
            } else if (std::abs(x) == 0.0) {
                cc = 0.0;
                ss = std::conj(y) / r;
            } else {
                cc = std::abs(x) / r;
                ss = (x / std::abs(x)) * std::conj(y) / r;
            }
            cs[k] = cc;
            sn[k] = ss;
            for (int j = k; j < m; ++j) {
                const cd u = H[k][j], w = H[k + 1][j];
                H[k][j] = cc * u + ss * w;
                H[k + 1][j] = -std::conj(ss) * u + cc * w;
            }
        }
        for (int k = lo; k < hi; ++k) {  // R Q: the same rotations from the right, and into Z
            const double cc = cs[k];
            const cd ss = sn[k];
            const int top = std::min(k + 2, hi);
            for (int i = 0; i <= top; ++i) {
                const cd u = H[i][k], w = H[i][k + 1];
                H[i][k] = cc * u + std::conj(ss) * w;
                H[i][k + 1] = -ss * u + cc * w;
            }
            for (int i = 0; i < m; ++i) {
                const cd u = Z[i][k], w = Z[i][k + 1];
                Z[i][k] = cc * u + std::conj(ss) * w;
                Z[i][k + 1] = -ss * u + cc * w;
            }
        }
        for (int i = lo; i <= hi; ++i) H[i][i] += mu;
    }
    return true;
}

// Time factor of the block systems of one direction with c_0 eliminated.  Per
// point the constraint sum_n s_n dc_n = sigma (s_n = (-1)^n) fixes dc_0 = sigma -
// sum_{j>=1} s_j dc_j, so the unknowns of a block mode are x = (dlam, dc_1 ..
// dc_{nt-1}) and its nt rows read M_r(e) x = rho - sigma K(e) e_0 with
//   K(e) = M0c - e U - zf W
// (M0c: the time coupling, i 2 on (m, k), k > m, k - m odd; adjoint: its
// conjugate transpose; W: the field's time matrix of the step, taken at the
// dipole coordinate zf; W = null for no field) and
//   M_r(e)[:, 0] = s,   M_r(e)[:, j] = K(e)[:, j] - s_j K(e)[:, 0]   (j >= 1).
// Split M_r(e) = M_r0 - e D_r (D_r[:, 0] = 0, D_r[:, j] = U_j e_j - s_j U_0 e_0)
// and diagonalise G = M_r0^{-1} D_r = S diag(lam) S^{-1}.  G's first column is
// zero, so e_0 is an eigenvector with eigenvalue 0 and the others come from the
// trailing block G22: for G22 u = lam u (lam != 0) the eigenvector of G is
// (g12 . u / lam, u) with g12 = G[0, 1..].  With simple eigenvalues
//   M_r(e)^{-1} = S (I - e diag(lam))^{-1} S^{-1} M_r0^{-1}.
// Outputs (row-major, nt x nt complex): E3 = S, E1 = S^{-1} M_r0^{-1}, and lam.
// Returns false if an eigenvalue of G22 is zero or repeated or G S = S diag(lam)
// fails to 1e-12.
bool time_factor(int nt, const double* U, const double* W, double zf, bool adjoint, cd* E1, cd* E3, cd* lam) {
    const int n = nt;
    cd K0[kTN][kTN], Mr0[kTN][kTN], Dr[kTN][kTN], Minv[kTN][kTN], G[kTN][kTN];
    for (int m = 0; m < n; ++m)
        for (int k = 0; k < n; ++k) {
            K0[m][k] = 0.0;
            Dr[m][k] = 0.0;
        }
    for (int m = 0; m < n; ++m)
        for (int k = 0; k < n; ++k) {
            if (k > m && ((k - m) & 1)) {
                if (!adjoint) K0[m][k] += cd(0.0, 2.0);
                else K0[k][m] += cd(0.0, -2.0);
            }
            if (W) K0[m][k] -= zf * W[m * n + k];
        }
    auto sgn = [](int j) { return (j & 1) ? -1.0 : 1.0; };
    for (int m = 0; m < n; ++m) {
        Mr0[m][0] = sgn(m);
        for (int j = 1; j < n; ++j) Mr0[m][j] = K0[m][j] - sgn(j) * K0[m][0];
    }
    for (int j = 1; j < n; ++j) {
        Dr[j][j] += U[j];
        Dr[0][j] -= sgn(j) * U[0];
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Minv[i][j] = Mr0[i][j];
    if (!invert_small(n, Minv)) return false;
    double gn = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cd acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Minv[i][k] * Dr[k][j];
            G[i][j] = acc;
            gn = std::max(gn, std::abs(acc));
        }
    cd S[kTN][kTN], lv[kTN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) S[i][j] = (i == j && j == 0) ? 1.0 : 0.0;
    lv[0] = 0.0;
    const int m = n - 1;
    if (m > 0) {
        cd T[kTN][kTN], Z[kTN][kTN];
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) T[i][j] = G[i + 1][j + 1];
        if (!schur_small(m, T, Z)) return false;
        for (int k = 0; k < m; ++k) {
            const cd lk = T[k][k];
            if (!(std::abs(lk) > 1e-12 * std::max(gn, 1e-300))) return false;
            cd w[kTN];
            for (int i = 0; i < m; ++i) w[i] = 0.0;
            w[k] = 1.0;
            for (int i = k - 1; i >= 0; --i) {
                cd acc = 0.0;
                for (int j = i + 1; j <= k; ++j) acc += T[i][j] * w[j];
                const cd den = T[i][i] - lk;
                if (std::abs(den) < 1e-12 * std::max(std::abs(lk), std::abs(T[i][i]))) return false;
                w[i] = -acc / den;
            }
            cd v[kTN];
            cd g12u = 0.0;
            for (int i = 0; i < m; ++i) {
                cd acc = 0.0;
                for (int j = 0; j <= k; ++j) acc += Z[i][j] * w[j];
                v[i + 1] = acc;
            }
            for (int i = 0; i < m; ++i) g12u += G[0][i + 1] * v[i + 1];
            v[0] = g12u / lk;
            double nv = 0.0;
            for (int i = 0; i < n; ++i) nv += std::norm(v[i]);
            nv = std::sqrt(nv);
            for (int i = 0; i < n; ++i) S[i][k + 1] = v[i] / nv;
            lv[k + 1] = lk;
        }
    }
    // check G S = S diag(lam)
    double err = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            cd gs = 0.0;
            for (int k = 0; k < n; ++k) gs += G[i][k] * S[k][j];
            err = std::max(err, std::abs(gs - S[i][j] * lv[j]));
        }
    if (!(err <= 1e-12 * std::max(gn, 1.0))) return false;
    cd Sinv[kTN][kTN];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Sinv[i][j] = S[i][j];
    if (!invert_small(n, Sinv)) return false;
    for (int i = 0; i < n; ++i) {
        lam[i] = lv[i];
        for (int j = 0; j < n; ++j) {
            E3[i * n + j] = S[i][j];
            cd acc = 0.0;
            for (int k = 0; k < n; ++k) acc += Sinv[i][k] * Minv[k][j];
            E1[i * n + j] = acc;
        }
    }
    return true;
}

void legendre_values(int nt, double y, double* P) {
    P[0] = 1.0;
    if (nt > 1) P[1] = y;
    for (int k = 1; k + 1 < nt; ++k) P[k + 1] = ((2.0 * k + 1.0) * y * P[k] - k * P[k - 1]) / (k + 1.0);
}

}  // namespace

struct lam_ctx {
    lam_grid grid{};
    lam_time time{};
    lam_ham ham{};
    lam_solver solver{};
    hipStream_t st = nullptr;
    int nt = 0;
    int L = 0;
    std::vector<Level> lv;
    std::vector<double> coef;
    double U[kMaxNT] = {};        // U_mm of the current step length dt_cur
    // time-step splitting: steps in progress have length dt_cur = dt / 2^depth
    int depth = 0;
    double dt_cur = 0.0;
    int state_depth = 0;          // depth of the state loaded in the context
    std::vector<double2*> d_split; // per depth: the state between two halves, then the
                                   // adjoint right-hand side between them (2P each)
    // current step
    double t0 = NAN;
    int W_depth = 0;              // depth whose step length W was built for
    double W[kMaxNT * kMaxNT] = {};
    int field_on = 0;
    int n_inner = 0;
    int have_state = 0;
    int adjoint = 0;
    double2* d_g = nullptr;       // adjoint: dL/dpsi_out^* (broadcast right-hand side)
    // reductions
    double* d_partial = nullptr;
    int max_parts = 0;
    double* d_red = nullptr;
    double* h_red = nullptr;      // pinned, mapped: the norm reduction writes it directly
    double* h_red_dev = nullptr;  // its device-side address
    hipEvent_t ev_norm = nullptr; // completion of the latest norm reduction
    double* h_norms = nullptr;    // pinned, mapped: N after each queued V-cycle of a solve (slot 0: N0)
    double* h_norms_dev = nullptr;
    int predict[2] = {0, 0};      // V-cycles the last forward / adjoint solve needed (0: none yet)
    // lam_propagate: the next step's initial state, built while the host waits
    // for the norms of the current step's last V-cycles (finest level)
    double2* d_c_next = nullptr;
    double2* d_lam_next = nullptr;
    double2* d_bs_next = nullptr;
    int solves[2] = {0, 0};       // forward / adjoint solves done
    double2* d_Gpart = nullptr;
    double2* d_G = nullptr;
    double2* h_G = nullptr;       // pinned
    double2* d_cf = nullptr;      // forward coefficients kept for the gradients
    // time factor records (layout in lam_internal.h): TS reals each
    int TS = 0;
    double* d_tf0 = nullptr;      // without field, per depth 0..max_split: the forward record,
                                  // then the adjoint one (FP64)
    float* d_tf0f = nullptr;      // and their FP32 copies
    std::vector<std::vector<double>> h_tf0;  // host copies, [2 depth + dir] (the fallback of a slab factor)
    size_t nslab_total = 0;       // slabs over all levels
    // with a field: per direction, one record per slab of every level (FP64), then
    // their FP32 copies; rebuilt on the host for every step and copied in stream order
    unsigned char* d_tfs[2] = {nullptr, nullptr};
    double tf_t[2] = {NAN, NAN};  // step (start, depth) whose records d_tfs[dir] hold
    int tf_depth[2] = {0, 0};
    double mf_t = NAN;            // stored per-mode inverses: step with a field they were built
    int mf_depth = 0;             // for (-inf: without field; NaN: none), and its depth
    struct Stage {                // pinned host staging of one step's records
        unsigned char* h = nullptr;
        hipEvent_t ev = nullptr;  // recorded after the copy that reads h
        double t = NAN;
        int dir = -1;
        int depth = 0;
    } stage[2];
    int stage_next = 0;
    double prep_t = NAN;          // a step whose records the next wait should prepare on the host
    int prep_dir = 0;
    double state_t0 = NAN;        // step of the state loaded in the context
    // iterated coarsest-level solve
    CoarseCtl* d_ctl = nullptr;
    int* h_citers = nullptr;      // pinned, mapped: per queued V-cycle, coarsest sweeps run | reached << 30
    int* h_citers_dev = nullptr;
    int coarse_launch = 0;        // coarsest iterations queued per V-cycle (learned; at most nu_coarse)
    int coarse_sweeps = 0;        // coarsest full sweeps run / V-cycles whose coarsest solve missed its
    int coarse_unmet = 0;         // reduction, since the current call started
    // adaptive tree: the finest level refined on some subvolumes (lam_set_refinement)
    bool refined = false;
    bool refine_off = false;      // lam_adjoint_step solves the unrefined step
    unsigned char* d_bmask = nullptr;   // one flag per finest subvolume
    int* d_act[2] = {nullptr, nullptr}; // the refined subvolumes of each colour
    int nact[2] = {0, 0};
    // profiling of finest-level sweeps
    int prof = 0;                 // record every prof-th finest-level sweep launch (0: off)
    long prof_count = 0;
    std::vector<hipEvent_t> ev;
    int nev = 0;
    int sweeps_fine = 0;
    double t_factor_ms = 0.0;
};

namespace {

// E(t) of the pulse h with Fourier amplitudes coef[0..ncoef).
double field_value(const lam_ham& h, const double* coef, int ncoef, double t) {
    if (h.pulse_kind == LAM_PULSE_NONE) return 0.0;
    if (t < 0.0 || t > h.t_total) return 0.0;
    double e = 0.0;
    if (h.pulse_kind == LAM_PULSE_SIN2 || h.pulse_kind == LAM_PULSE_SIN2_FOURIER) {
        const double s = std::sin(M_PI * t / h.t_total);
        e += h.e0 * s * s * std::cos(h.omega * t);
    }
    if (h.pulse_kind == LAM_PULSE_FOURIER || h.pulse_kind == LAM_PULSE_SIN2_FOURIER) {
        for (int q = 0; q < ncoef; ++q) e += coef[q] * std::sin((q + 1) * M_PI * t / h.t_total);
    }
    return e;
}

// W_nm = int_{t0}^{t0+dt} T_n T_m f(t) dt for f = E (q < 0) or the q-th sine.
void time_matrix(const lam_ham& h, const double* coef, int ncoef, int nt, double dt, double t0, int q,
                 double* W) {
    const GaussNodes& gl = gauss_nodes();
    for (int k = 0; k < nt * nt; ++k) W[k] = 0.0;
    double P[kMaxNT];
    for (int k = 0; k < kGL; ++k) {
        const double t = t0 + 0.5 * dt * (gl.x[k] + 1.0);
        double f;
        if (q < 0) {
            f = field_value(h, coef, ncoef, t);
        } else {
            f = (t < 0.0 || t > h.t_total) ? 0.0 : std::sin((q + 1) * M_PI * t / h.t_total);
        }
        if (f == 0.0) continue;
        legendre_values(nt, gl.x[k], P);
        const double wk = 0.5 * dt * gl.w[k] * f;
        for (int n = 0; n < nt; ++n)
            for (int m = 0; m < nt; ++m) W[n * nt + m] += wk * P[n] * P[m];
    }
}

void time_matrix(const lam_ctx* c, double t0, int q, double* W) {
    time_matrix(c->ham, c->coef.data(), (int)c->coef.size(), c->nt, c->dt_cur, t0, q, W);
}

bool any_nonzero(const double* W, int n) {
    for (int k = 0; k < n; ++k)
        if (W[k] != 0.0) return true;
    return false;
}

// Real form (2n x 2n, acting on interleaved re/im) of an n x n complex matrix.
void real_form(int n, const cd* M, double* out) {
    const int n2 = 2 * n;
    for (int r = 0; r < n2; ++r)
        for (int q = 0; q < n2; ++q) {
            const cd m = M[(r >> 1) * n + (q >> 1)];
            const int a = r & 1, cc = q & 1;
            out[r * n2 + q] = (a == cc) ? m.real() : (a == 0 ? -m.imag() : m.imag());
        }
}

// One time factor record (layout in lam_internal.h) of direction dir with the
// field's time matrix W (null: none) taken at zf.  false if the factor fails.
bool make_record(const lam_ctx* c, const double* W, double zf, int dir, double* rec) {
    const int n = c->nt;
    cd E1[kTN * kTN], E3[kTN * kTN], lam[kTN];
    if (!time_factor(n, c->U, W, zf, dir != 0, E1, E3, lam)) return false;
    real_form(n, E1, rec);
    real_form(n, E3, rec + 4 * n * n);
    for (int k = 0; k < n; ++k) {
        rec[8 * n * n + 2 * k] = lam[k].real();
        rec[8 * n * n + 2 * k + 1] = lam[k].imag();
    }
    rec[tf_record_reals(n)] = zf;
    rec[tf_record_reals(n) + 1] = 0.0;
    return true;
}

size_t tf_table_bytes(const lam_ctx* c) { return c->nslab_total * (size_t)c->TS * (sizeof(double) + sizeof(float)); }

// Build on the host the records of step t (direction dir) for every slab of
// every level, into a staging buffer (reused if it already holds them).  A
// slab whose factor fails takes the record without field (zf = 0), so its
// inner passes correct the whole field term.
int prepare_tables(lam_ctx* c, double t, int dir) {
    for (auto& s : c->stage)
        if (s.t == t && s.dir == dir && s.depth == c->depth) return LAM_OK;
    auto& s = c->stage[c->stage_next];
    c->stage_next ^= 1;
    HIPCHK(hipEventSynchronize(s.ev));  // the copy that last read this buffer is done
    s.t = NAN;
    double W[kMaxNT * kMaxNT];
    time_matrix(c, t, -1, W);
    const int TS = c->TS;
    double* h64 = reinterpret_cast<double*>(s.h);
    float* h32 = reinterpret_cast<float*>(s.h + c->nslab_total * (size_t)TS * sizeof(double));
    for (const auto& L : c->lv)
        for (int k = 0; k < L.nslab; ++k) {
            double* rec = h64 + (L.tf_off + k) * (size_t)TS;
            if (!make_record(c, W, L.zslab[k], dir, rec)) {
                const auto& fb = c->h_tf0[2 * c->depth + dir];
                std::copy(fb.begin(), fb.end(), rec);
            }
            float* rf = h32 + (L.tf_off + k) * (size_t)TS;
            for (int i = 0; i < TS; ++i) rf[i] = (float)rec[i];
        }
    s.t = t;
    s.dir = dir;
    s.depth = c->depth;
    return LAM_OK;
}

// Make d_tfs[dir] hold the records of step t (a copy queued on the stream:
// kernels queued before it still read the previous records).
int upload_tables(lam_ctx* c, double t, int dir) {
    if (c->tf_t[dir] == t && c->tf_depth[dir] == c->depth) return LAM_OK;
    LAMCHK(prepare_tables(c, t, dir));
    for (auto& s : c->stage)
        if (s.t == t && s.dir == dir && s.depth == c->depth) {
            HIPCHK(hipMemcpyAsync(c->d_tfs[dir], s.h, tf_table_bytes(c), hipMemcpyHostToDevice, c->st));
            HIPCHK(hipEventRecord(s.ev, c->st));
            c->tf_t[dir] = t;
            c->tf_depth[dir] = c->depth;
            return LAM_OK;
        }
    return LAM_EINVAL;
}

// Stored per-mode inverses (LAM_TF_STORED) for the current step: with the
// field at each slab's zf (records of direction dir), or without field.
int stored_factors(lam_ctx* c, int dir) {
    if (c->solver.time_factor != LAM_TF_STORED) return LAM_OK;
    const double want = c->field_on ? c->t0 : -INFINITY;
    if (c->mf_t == want && c->mf_depth == c->depth) return LAM_OK;
    for (auto& L : c->lv) {
        const double* tf = c->field_on ? reinterpret_cast<const double*>(c->d_tfs[dir]) + L.tf_off * (size_t)c->TS
                                       : nullptr;
        HIPCHK(launch_mode_factor(c->nt, L.g, c->U, c->field_on ? c->W : nullptr, L.d_e, tf, c->TS, L.d_Minv,
                                  L.fp32 ? L.d_Minvf : nullptr, c->st));
    }
    c->mf_t = want;
    c->mf_depth = c->depth;
    return LAM_OK;
}

// Steps of length dt / 2^d from now on (U and, through the step length, every
// field matrix and time factor record; the records without field are kept per
// depth, the others are rebuilt on demand, keyed by their depth).
void set_depth(lam_ctx* c, int d) {
    if (c->depth == d && c->dt_cur > 0.0) return;
    c->depth = d;
    c->dt_cur = std::ldexp(c->time.dt, -d);
    for (int m = 0; m < c->nt; ++m) c->U[m] = c->dt_cur / (2.0 * m + 1.0);
}

// Select the step starting at t0 for solves of direction dir (0 forward, 1
// adjoint): its field matrix, inner-pass count and time factor records.
int set_step(lam_ctx* c, double t0, int dir) {
    if (!(c->t0 == t0 && c->W_depth == c->depth)) {
        time_matrix(c, t0, -1, c->W);
        c->t0 = t0;
        c->W_depth = c->depth;
    }
    const int nt = c->nt;
    const bool on = any_nonzero(c->W, nt * nt);
    c->field_on = on;
    c->n_inner = c->solver.n_inner >= 0 ? c->solver.n_inner : (on ? 16 : 0);
    auto t_a = std::chrono::steady_clock::now();
    if (on) LAMCHK(upload_tables(c, t0, dir));
    LAMCHK(stored_factors(c, dir));
    c->t_factor_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_a).count();
    return LAM_OK;
}

// Whether the step starting at t0 sees a field (its time matrix is nonzero); W (may be null) receives it.
bool step_field(const lam_ctx* c, double t0, double* W) {
    double Wl[kMaxNT * kMaxNT];
    double* w = W ? W : Wl;
    time_matrix(c, t0, -1, w);
    return any_nonzero(w, c->nt * c->nt);
}

int factor_level(lam_ctx* c, Level& L) {
    HIPCHK(launch_block_eig(L.g, L.d_v0, L.d_V, L.d_e, L.fp32 ? L.d_Vf : nullptr, c->st));
    c->mf_t = NAN;  // stored per-mode inverses depend on the eigenvalues
    return LAM_OK;
}

// Whether solves use the adaptive tree now (forward solves with a refinement set).
bool refining(const lam_ctx* c) { return c->refined && !c->refine_off && !c->adjoint; }

// Partials of N for the context state into d_partial; *np receives their count.
// With the adaptive tree: the refined rows of the finest residual plus the
// projected residual on level 1 (written into level 1's right-hand side, which
// the next V-cycle overwrites anyway).
int norm_partials(lam_ctx* c, int* np) {
    Level& L = c->lv[0];
    const double2* bg = c->adjoint ? c->d_g : nullptr;
    const double2* bs = c->adjoint ? nullptr : L.d_bs;
    const bool comp = refining(c);
    HIPCHK(launch_residual(c->nt, L.g, c->U, c->W, c->adjoint, c->field_on, L.d_c, L.d_lam, L.d_v0, nullptr, bg, bs,
                           nullptr, nullptr, c->d_partial, np, c->st, nullptr, comp ? c->d_bmask : nullptr));
    if (comp) {
        Level& C = c->lv[1];
        HIPCHK(launch_residual_restrict(c->nt, L.g, C.g, c->U, c->W, c->adjoint, c->field_on, L.d_c, L.d_lam,
                                        L.d_v0, nullptr, bg, bs, C.d_bc, C.d_bs, C.d_c, C.d_lam, c->st));
        int np2 = 0;
        HIPCHK(launch_rhs_norm(c->nt, C.g.P, c->U, C.d_bc, C.d_bs, c->d_partial + *np, &np2, c->st));
        *np += np2;
    }
    return LAM_OK;
}

int sweep(lam_ctx* c, int l, int colour, const int* skip = nullptr) {
    Level& L = c->lv[l];
    SweepArgs a{};
    a.skip = skip;
    a.g = L.g;
    a.blocks = L.d_blocks[colour];
    a.colour = colour;
    a.arith_blocks = (L.g.nblk[L.g.dim - 1] % 2 == 0) ? 1 : 0;
    a.half_last = std::max(1, L.g.nblk[L.g.dim - 1] / 2);
    int nblk = L.ncol[colour];
    if (l == 0 && refining(c)) {
        // adaptive tree: only the refined subvolumes of the colour
        a.blocks = c->d_act[colour];
        a.arith_blocks = 0;
        nblk = c->nact[colour];
    }
    a.c = L.d_c;
    a.lam = L.d_lam;
    a.v0 = L.d_v0;
    if (l == 0) {
        a.bc = nullptr;
        a.bg = c->adjoint ? c->d_g : nullptr;
        a.bs = c->adjoint ? nullptr : L.d_bs;
    } else {
        a.bc = L.d_bc;
        a.bg = nullptr;
        a.bs = L.d_bs;
    }
    a.V = L.fp32 ? static_cast<const void*>(L.d_Vf) : static_cast<const void*>(L.d_V);
    if (c->solver.time_factor == LAM_TF_STORED)
        a.Minv = L.fp32 ? static_cast<const void*>(L.d_Minvf) : static_cast<const void*>(L.d_Minv);
    else
        a.Minv = nullptr;
    const int dir = c->adjoint ? 1 : 0;
    if (c->field_on) {
        const size_t off = L.tf_off * (size_t)c->TS;
        const double* t64 = reinterpret_cast<const double*>(c->d_tfs[dir]);
        const float* t32 = reinterpret_cast<const float*>(c->d_tfs[dir] + c->nslab_total * (size_t)c->TS * sizeof(double));
        a.tf = L.fp32 ? static_cast<const void*>(t32 + off) : static_cast<const void*>(t64 + off);
        a.tf_stride = c->TS;
    } else {
        const size_t off = (2 * (size_t)c->depth + dir) * c->TS;
        a.tf = L.fp32 ? static_cast<const void*>(c->d_tf0f + off) : static_cast<const void*>(c->d_tf0 + off);
        a.tf_stride = 0;
    }
    a.e = L.d_e;
    a.passes = L.d_passes;
    a.adjoint = c->adjoint;
    a.n_inner = c->n_inner;
    {
        const double tol = c->solver.inner_tol > 0.0 ? c->solver.inner_tol : 1e-2;
        a.inner_tol2 = tol * tol;
        // ||W||_2 <= max_m sum_n |W_mn| for the symmetric field matrix
        double wb = 0.0;
        for (int m = 0; m < c->nt && c->field_on; ++m) {
            double r = 0.0;
            for (int n = 0; n < c->nt; ++n) r += std::fabs(c->W[m * c->nt + n]);
            wb = std::max(wb, r);
        }
        a.wbound2 = wb * wb;
    }
    a.field_on = c->field_on ? 1 : 0;
    const bool rec = c->prof > 0 && l == 0 && (c->prof_count++ % c->prof) == 0;
    if (rec) {
        while ((int)c->ev.size() < c->nev + 2) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            c->ev.push_back(e);
        }
        HIPCHK(hipEventRecord(c->ev[c->nev], c->st));
    }
    HIPCHK(launch_sweep(c->nt, L.fp32 ? 1 : 0, a, c->U, c->W, nblk, c->st));
    if (rec) {
        HIPCHK(hipEventRecord(c->ev[c->nev + 1], c->st));
        c->nev += 2;
    }
    return LAM_OK;
}

int full_sweep(lam_ctx* c, int l, const int* skip = nullptr) {
    LAMCHK(sweep(c, l, 0, skip));
    LAMCHK(sweep(c, l, 1, skip));
    if (l == 0) c->sweeps_fine++;
    return LAM_OK;
}

// The coarsest-level solve of a V-cycle (Eq. (correction_fine): the coarse
// correction solves the coarse system for the projected residual).  Without a
// reduction target: exactly nu_coarse full sweeps.  With one (solver
// coarse_reduction > 0): full sweeps until the coarsest residual norm has
// fallen by that factor, at most nu_coarse.  The decision is taken on the
// device: after each full sweep a residual and its sum update the control
// block, and once the target is reached the remaining queued launches of the
// solve do nothing.  The host queues as many iterations as the previous
// V-cycles needed plus one (at most nu_coarse), learning from the counts the
// reductions leave in mapped host memory (slot: this V-cycle's, -1 for none).
int coarsest_solve(lam_ctx* c, int l, int slot) {
    const double red = c->solver.coarse_reduction;
    if (!(red > 0.0)) {
        for (int s = 0; s < c->grid.nu_coarse; ++s) LAMCHK(full_sweep(c, l));
        return LAM_OK;
    }
    Level& L = c->lv[l];
    const double2* bc = l == 0 ? nullptr : L.d_bc;
    const double2* bg = (l == 0 && c->adjoint) ? c->d_g : nullptr;
    const double2* bs = (l == 0 && c->adjoint) ? nullptr : L.d_bs;
    const int* done = &c->d_ctl->done;
    int np = 0;
    HIPCHK(launch_residual(c->nt, L.g, c->U, c->W, c->adjoint, c->field_on, L.d_c, L.d_lam, L.d_v0, bc, bg, bs,
                           nullptr, nullptr, c->d_partial, &np, c->st));
    HIPCHK(launch_reduce_ctl(c->d_partial, np, c->d_ctl, 1, 0.0, nullptr, c->st));
    const int n_it = std::min(c->grid.nu_coarse, std::max(1, c->coarse_launch));
    for (int it = 0; it < n_it; ++it) {
        LAMCHK(full_sweep(c, l, done));
        HIPCHK(launch_residual(c->nt, L.g, c->U, c->W, c->adjoint, c->field_on, L.d_c, L.d_lam, L.d_v0, bc, bg, bs,
                               nullptr, nullptr, c->d_partial, &np, c->st, done));
        HIPCHK(launch_reduce_ctl(c->d_partial, np, c->d_ctl, 0, red * red,
                                 (it == n_it - 1 && slot >= 0) ? c->h_citers_dev + slot : nullptr, c->st));
    }
    return LAM_OK;
}

// Account for the coarsest solves of V-cycles [first, last] (their slots).
void note_coarsest(lam_ctx* c, int first, int last) {
    if (!(c->solver.coarse_reduction > 0.0)) return;
    int used = 0;
    for (int k = first; k <= last; ++k) {
        const int v = c->h_citers[k];
        const int it = v & 0x3fffffff;
        const bool met = (v >> 30) & 1;
        c->coarse_sweeps += it;
        if (!met) c->coarse_unmet++;
        // a solve that ran every queued iteration without reaching the target asks for all
        used = std::max(used, met ? it : c->grid.nu_coarse);
    }
    c->coarse_launch = std::min(c->grid.nu_coarse, used + 1);
}

// Wait for the work queued on the context stream (e.g. a norm reduction that
// writes host memory): an event polled in a loop, so the host resumes as soon
// as the work is done (a blocking stream synchronisation can add tens of
// microseconds of wake-up latency to every V-cycle).  wait_event polls
// ev_norm as recorded earlier; wait_stream records it at the end of the queue.
int wait_event(lam_ctx* c) {
    for (;;) {
        const hipError_t e = hipEventQuery(c->ev_norm);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) return LAM_EHIP;
    }
    return LAM_OK;
}

int wait_stream(lam_ctx* c) {
    HIPCHK(hipEventRecord(c->ev_norm, c->st));
    return wait_event(c);
}

// N of the finest level for the context state (synchronises).
int norm0(lam_ctx* c, double* out) {
    int np = 0;
    LAMCHK(norm_partials(c, &np));
    HIPCHK(launch_reduce(c->d_partial, np, 1, c->h_red_dev, c->st));
    LAMCHK(wait_stream(c));
    *out = c->h_red[0];
    return LAM_OK;
}

int vcycle(lam_ctx* c, int l, int slot = -1) {
    if (l == c->L - 1) return coarsest_solve(c, l, slot);
    for (int s = 0; s < c->grid.nu_pre; ++s) LAMCHK(full_sweep(c, l));
    Level& F = c->lv[l];
    Level& C = c->lv[l + 1];
    // residual of level l restricted into the right-hand side of level l + 1,
    // whose correction starts from zero
    const double2* bc = l == 0 ? nullptr : F.d_bc;
    const double2* bg = (l == 0 && c->adjoint) ? c->d_g : nullptr;
    const double2* bs = (l == 0 && c->adjoint) ? nullptr : F.d_bs;
    HIPCHK(launch_residual_restrict(c->nt, F.g, C.g, c->U, c->W, c->adjoint, c->field_on, F.d_c, F.d_lam, F.d_v0, bc,
                                    bg, bs, C.d_bc, C.d_bs, C.d_c, C.d_lam, c->st));
    LAMCHK(vcycle(c, l + 1, slot));
    HIPCHK(launch_prolong(c->nt, F.g, C.g, c->grid.interp, C.d_c, C.d_lam, F.d_c, F.d_lam, c->st));
    for (int s = 0; s < c->grid.nu_post; ++s) LAMCHK(full_sweep(c, l));
    return LAM_OK;
}

// V-cycles on the context state until sqrt(N/N0) <= tol.
// Queue N of the finest level for the context state into h_norms[slot] (no wait).
int queue_norm(lam_ctx* c, int slot) {
    int np = 0;
    LAMCHK(norm_partials(c, &np));
    HIPCHK(launch_reduce(c->d_partial, np, 1, c->h_norms_dev + slot, c->st));
    return LAM_OK;
}

// V-cycles until sqrt(N/N0) <= tol.  The cycles are queued in batches: as many
// as the previous solve of the same kind needed (none before the first wait of
// a context's first solve), the last two followed by their norms (written to
// host memory), then one wait; after that one cycle per wait.  A
// host round trip per cycle would leave the GPU idle while the next cycle is
// launched.  When a batch overshoots, the extra cycles only refine the state;
// `cycles` reports the cycles run.
// n0_slot >= 0: N0 of this (forward) solve is already queued into that slot.
// While the step may still be split (depth < max_split), a solve whose checked
// norm ends above N0, or above the norm checked before it while still far from
// tol (above 100 tol, clear of the rounding floor), is abandoned at once
// (LAM_EDIVERGED): it is leaving the convergent regime, and the shorter steps
// will be solved instead.
// next_out non-null (forward solves of lam_propagate whose next step has no
// field, like this one): before each wait, the end state goes to next_out, the
// next step's initial state to the context's d_*_next buffers and its N0 to
// h_norms[next_slot], so that the GPU has work while the host reacts to the
// norms; *next_ready tells whether that was done after the final cycle.
int solve_loop(lam_ctx* c, lam_stats* stats, int n0_slot = -1, double2* next_out = nullptr, int next_slot = 0,
               bool* next_ready = nullptr, const double* next_W = nullptr) {
    const int maxc = c->solver.max_cycles;
    int& predict = c->predict[c->adjoint ? 1 : 0];
    if (next_ready) *next_ready = false;
    if (n0_slot < 0) {
        n0_slot = 0;
        LAMCHK(queue_norm(c, 0));
    }
    int queued = 0, conv = -1;
    int rc = LAM_ENOCONV;
    int batch = std::min(predict, maxc);  // 0 on a context's first solve: look at N0 first
    const int cs0 = c->coarse_sweeps, cu0 = c->coarse_unmet;
    const bool may_split = c->depth < c->solver.max_split;
    double N0 = 0.0, N = 0.0, Nchk = -1.0;
    for (;;) {
        const int nb = std::min(batch, maxc - queued);
        // norms after the last cycle of the batch (it decides) and, on every
        // eighth solve of this kind, after the one before (whether the next solves
        // can use one cycle less)
        const bool probe = (c->solves[c->adjoint ? 1 : 0] & 7) == 0;
        int first_norm = -1;   // the first cycle of this batch whose norm is queued
        for (int i = 0; i < nb; ++i) {
            LAMCHK(vcycle(c, 0, queued + 1));
            ++queued;
            if (i == nb - 1 || (probe && i == nb - 2)) {
                LAMCHK(queue_norm(c, queued));
                if (first_norm < 0) first_norm = queued;
            }
        }
        // the host waits for the norms only; queued after them, the next
        // step's start keeps the GPU busy while the host reacts
        HIPCHK(hipEventRecord(c->ev_norm, c->st));
        if (next_out) {
            Level& L = c->lv[0];
            int np = 0;
            HIPCHK(launch_advance(c->nt, L.g, c->U, next_W, L.d_c, L.d_v0, next_out, c->d_c_next, c->d_lam_next,
                                  c->d_bs_next, c->d_partial, &np, c->st));
            HIPCHK(launch_reduce(c->d_partial, np, 1, c->h_norms_dev + next_slot, c->st));
        }
        // the host builds the next step's time factor records while the GPU works
        if (!std::isnan(c->prep_t)) {
            const double tp = c->prep_t;
            c->prep_t = NAN;
            LAMCHK(prepare_tables(c, tp, c->prep_dir));
        }
        LAMCHK(wait_event(c));
        if (nb > 0) note_coarsest(c, queued - nb + 1, queued);
        N0 = c->h_norms[n0_slot];
        N = c->h_norms[queued];
        if (!std::isfinite(N0)) {
            rc = LAM_EDIVERGED;
            break;
        }
        if (N0 == 0.0) {
            rc = LAM_OK;
            if (next_ready) *next_ready = next_out != nullptr;
            break;
        }
        bool div = false;
        if (Nchk < 0.0) Nchk = N0;
        for (int k = first_norm; first_norm >= 0 && k <= queued; ++k) {
            const double Nk = c->h_norms[k];
            if (!std::isfinite(Nk) || Nk > 1e12 * N0) {
                div = true;
                break;
            }
            if (may_split && (Nk > N0 || (Nk > Nchk && std::sqrt(Nk / N0) > 100.0 * c->solver.tol))) {
                div = true;
                break;
            }
            Nchk = Nk;
            if (conv < 0 && std::sqrt(Nk / N0) <= c->solver.tol) conv = k;
        }
        if (div) {
            rc = LAM_EDIVERGED;
            break;
        }
        if (conv >= 0) {
            rc = LAM_OK;
            if (next_ready) *next_ready = next_out != nullptr;
            break;
        }
        if (queued >= maxc) break;
        batch = 1;
    }
    if (conv > 0) predict = conv;
    ++c->solves[c->adjoint ? 1 : 0];
    if (stats) {
        stats->cycles = queued;
        stats->resid0 = std::sqrt(N0);
        stats->resid = std::sqrt(N);
        stats->resid0_last = stats->resid0;
        stats->resid_last = stats->resid;
        stats->coarse_sweeps = c->coarse_sweeps - cs0;
        stats->coarse_unmet = c->coarse_unmet - cu0;
    }
    return rc;
}

bool bad_ptr(const void* p) { return p == nullptr; }

int validate(const lam_grid* g, const lam_time* t, const lam_ham* h, const lam_solver* s) {
    if (!g || !t || !h || !s) return LAM_EINVAL;
    if (g->dim < 1 || g->dim > 3) return LAM_EINVAL;
    if (!(g->h > 0.0) || !(t->dt > 0.0) || !(h->mass > 0.0)) return LAM_EINVAL;
    if (t->n_t < 1 || t->n_t > LAM_MAX_NT) return LAM_EINVAL;
    if (g->levels < 1 || g->levels > 16) return LAM_EINVAL;
    if (g->nu_pre < 0 || g->nu_post < 0 || g->nu_coarse < 0) return LAM_EINVAL;
    if (g->interp != 0 && g->interp != 1) return LAM_EINVAL;
    if (g->coarse_op != LAM_COARSE_REDISCRETISED && g->coarse_op != LAM_COARSE_GALERKIN) return LAM_EINVAL;
    if (g->coarse_op == LAM_COARSE_GALERKIN && g->interp != 1) return LAM_EINVAL;
    if (h->field_axis < 0 || h->field_axis >= g->dim) return LAM_EINVAL;
    if (h->pulse_kind < LAM_PULSE_NONE || h->pulse_kind > LAM_PULSE_SIN2_FOURIER) return LAM_EINVAL;
    if (h->pulse_kind != LAM_PULSE_NONE && !(h->t_total > 0.0)) return LAM_EINVAL;
    if (h->n_coef < 0 || (h->n_coef > 0 && !h->coef)) return LAM_EINVAL;
    if (!h->v0) return LAM_EINVAL;
    if (s->precision != LAM_FP64 && s->precision != LAM_MIXED) return LAM_EINVAL;
    if (s->max_cycles < 0 || !(s->tol >= 0.0) || s->n_inner < -1 || s->n_inner > LAM_MAX_INNER) return LAM_EINVAL;
    if (!(s->coarse_reduction >= 0.0 && s->coarse_reduction < 1.0)) return LAM_EINVAL;
    if (s->max_split < 0 || s->max_split > LAM_MAX_SPLIT) return LAM_EINVAL;
    if (!(s->inner_tol >= 0.0 && s->inner_tol < 1.0)) return LAM_EINVAL;
    if (s->time_factor != LAM_TF_SHARED && s->time_factor != LAM_TF_STORED) return LAM_EINVAL;
    long bpts = 1;
    for (int a = 0; a < g->dim; ++a) {
        if (g->n[a] < 1 || g->block[a] < 1) return LAM_EINVAL;
        bpts *= g->block[a];
        long n = g->n[a];
        for (int l = 0; l < g->levels; ++l) {
            if (n % g->block[a]) return LAM_EINVAL;
            const long nb = n / g->block[a];
            if (g->periodic && nb > 1 && (nb & 1)) return LAM_EINVAL;
            if (g->periodic && n < 2) return LAM_EINVAL;
            if (l + 1 < g->levels) {
                if (n & 1) return LAM_EINVAL;
                n /= 2;
            }
        }
    }
    if (bpts > LAM_MAX_BLOCK) return LAM_EINVAL;
    long P = 1;
    for (int a = 0; a < g->dim; ++a) {
        P *= g->n[a];
        if (P > (1L << 30)) return LAM_EINVAL;
    }
    return LAM_OK;
}

template <typename T>
int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) return LAM_OK;
    if (hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * count) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return LAM_ENOMEM;
    }
    return LAM_OK;
}

// The spare finest-level state of lam_propagate, allocated on first use: all
// three buffers or none (on failure the steps run without them).
bool alloc_next(lam_ctx* c) {
    if (c->d_c_next && c->d_lam_next && c->d_bs_next) return true;
    const size_t P = (size_t)c->lv[0].g.P;
    bool ok = dalloc(&c->d_c_next, P * c->nt) == LAM_OK;
    ok = ok && dalloc(&c->d_lam_next, P) == LAM_OK;
    ok = ok && dalloc(&c->d_bs_next, P) == LAM_OK;
    if (!ok) {
        (void)hipFree(c->d_c_next);
        (void)hipFree(c->d_lam_next);
        c->d_c_next = nullptr;
        c->d_lam_next = nullptr;
        c->d_bs_next = nullptr;
    }
    return ok;
}

void free_ctx(lam_ctx* c) {
    if (!c) return;
    if (c->st) (void)hipStreamSynchronize(c->st);
    for (auto& L : c->lv) {
        for (int k = 0; k < 2; ++k) (void)hipFree(L.d_blocks[k]);
        (void)hipFree(L.d_v0);
        (void)hipFree(L.d_c);
        (void)hipFree(L.d_lam);
        (void)hipFree(L.d_bc);
        (void)hipFree(L.d_bs);
        (void)hipFree(L.d_V);
        (void)hipFree(L.d_e);
        (void)hipFree(L.d_Vf);
        (void)hipFree(L.d_Minv);
        (void)hipFree(L.d_Minvf);
        (void)hipFree(L.d_passes);
    }
    (void)hipFree(c->d_g);
    (void)hipFree(c->d_partial);
    (void)hipFree(c->d_red);
    (void)hipFree(c->d_Gpart);
    (void)hipFree(c->d_G);
    (void)hipFree(c->d_cf);
    (void)hipFree(c->d_tf0);
    (void)hipFree(c->d_tf0f);
    for (auto* p : c->d_tfs) (void)hipFree(p);
    for (auto& s : c->stage) {
        if (s.h) (void)hipHostFree(s.h);
        if (s.ev) (void)hipEventDestroy(s.ev);
    }
    if (c->h_red) (void)hipHostFree(c->h_red);
    if (c->ev_norm) (void)hipEventDestroy(c->ev_norm);
    if (c->h_norms) (void)hipHostFree(c->h_norms);
    if (c->h_citers) (void)hipHostFree(c->h_citers);
    (void)hipFree(c->d_ctl);
    (void)hipFree(c->d_c_next);
    (void)hipFree(c->d_lam_next);
    (void)hipFree(c->d_bs_next);
    for (auto* p : c->d_split) (void)hipFree(p);
    (void)hipFree(c->d_bmask);
    for (auto* p : c->d_act) (void)hipFree(p);
    if (c->h_G) (void)hipHostFree(c->h_G);
    for (auto e : c->ev) (void)hipEventDestroy(e);
    delete c;
}

// Geometry of level l of a (validated) grid.
LevelGeom level_geom(const lam_grid& gr, const lam_ham& ham, int l) {
    LevelGeom g{};
    g.dim = gr.dim;
    g.P = 1;
    g.nblk[0] = g.nblk[1] = g.nblk[2] = 1;
    g.bdim[0] = g.bdim[1] = g.bdim[2] = 1;
    g.n[0] = g.n[1] = g.n[2] = 1;
    for (int a = 0; a < gr.dim; ++a) {
        g.n[a] = gr.n[a] >> l;
        g.bdim[a] = gr.block[a];
        g.nblk[a] = g.n[a] / g.bdim[a];
        g.P *= g.n[a];
    }
    g.h = gr.h * std::ldexp(1.0, l);
    g.periodic = gr.periodic;
    g.fax = ham.field_axis;
    // rediscretised: 1/(2 m H^2); Galerkin with piecewise-constant interpolation:
    // the finer level's coefficient halved, 1/(2 m h^2 2^l)
    g.kin = gr.coarse_op == LAM_COARSE_GALERKIN ? 1.0 / (2.0 * ham.mass * gr.h * gr.h * std::ldexp(1.0, l))
                                                : 1.0 / (2.0 * ham.mass * g.h * g.h);
    g.bpts = g.bdim[0] * g.bdim[1] * g.bdim[2];
    g.rbp = 1.0f / (float)g.bpts;
    for (int a = 0; a < 3; ++a) {
        g.rn[a] = 1.0 / g.n[a];
        g.rnb[a] = 1.0 / g.nblk[a];
        g.rbd[a] = 1.0f / (float)g.bdim[a];
    }
    return g;
}

int build(lam_ctx* c, const double* v0_dev) {
    const lam_grid& gr = c->grid;
    const int nt = c->nt;
    c->lv.resize(gr.levels);
    for (int l = 0; l < gr.levels; ++l) {
        Level& L = c->lv[l];
        LevelGeom& g = L.g;
        g = level_geom(gr, c->ham, l);
        L.nblocks = g.nblk[0] * g.nblk[1] * g.nblk[2];
        L.fp32 = c->solver.precision == LAM_MIXED && (l < gr.levels - 1 || gr.levels == 1);
        // colour lists
        std::vector<int> col[2];
        for (int b = 0; b < L.nblocks; ++b) {
            int bc[3] = {0, 0, 0}, t = b;
            for (int a = gr.dim - 1; a >= 0; --a) {
                bc[a] = t % g.nblk[a];
                t /= g.nblk[a];
            }
            col[(bc[0] + bc[1] + bc[2]) & 1].push_back(b);
        }
        // slabs of blocks along the field axis and their centre coordinates, rounded
        // to FP32 so that both precisions' factor records hold the same zf exactly
        {
            const int a = g.fax;
            L.nslab = g.nblk[a];
            L.zslab.resize(L.nslab);
            for (int k = 0; k < L.nslab; ++k) {
                const double centre_index = k * g.bdim[a] + 0.5 * (g.bdim[a] - 1);
                L.zslab[k] = (double)(float)((centre_index - 0.5 * (g.n[a] - 1)) * g.h);
            }
            L.tf_off = c->nslab_total;
            c->nslab_total += L.nslab;
        }
        for (int k = 0; k < 2; ++k) {
            L.ncol[k] = (int)col[k].size();
            LAMCHK(dalloc(&L.d_blocks[k], col[k].size()));
            if (!col[k].empty())
                HIPCHK(hipMemcpy(L.d_blocks[k], col[k].data(), sizeof(int) * col[k].size(),
                                 hipMemcpyHostToDevice));
        }
        const size_t P = g.P;
        const size_t B = g.bpts;
        LAMCHK(dalloc(&L.d_v0, P));
        LAMCHK(dalloc(&L.d_c, P * nt));
        LAMCHK(dalloc(&L.d_lam, P));
        LAMCHK(dalloc(&L.d_bs, P));
        if (l > 0) LAMCHK(dalloc(&L.d_bc, P * nt));
        LAMCHK(dalloc(&L.d_V, L.nblocks * B * B));
        LAMCHK(dalloc(&L.d_e, L.nblocks * B));
        const bool stored = c->solver.time_factor == LAM_TF_STORED;
        if (stored) LAMCHK(dalloc(&L.d_Minv, L.nblocks * B * (nt + 1) * (nt + 1)));
        LAMCHK(dalloc(&L.d_passes, (size_t)L.nblocks));
        HIPCHK(hipMemsetAsync(L.d_passes, 0, (size_t)L.nblocks, c->st));
        if (L.fp32) {
            LAMCHK(dalloc(&L.d_Vf, L.nblocks * B * B));
            if (stored) LAMCHK(dalloc(&L.d_Minvf, L.nblocks * B * (nt + 1) * (nt + 1)));
        }
    }
    HIPCHK(hipMemcpyAsync(c->lv[0].d_v0, v0_dev, sizeof(double) * c->lv[0].g.P, hipMemcpyDeviceToDevice, c->st));
    for (int l = 1; l < gr.levels; ++l)
        HIPCHK(launch_average_potential(c->lv[l - 1].g, c->lv[l].g, c->lv[l - 1].d_v0, c->lv[l].d_v0, c->st));
    const int P0 = c->lv[0].g.P;
    c->max_parts = (P0 + kThreads - 1) / kThreads;
    // norm partials: the finest level's, then (composite norm of the adaptive tree) level 1's
    LAMCHK(dalloc(&c->d_partial, (size_t)residual_blocks(nt, P0) +
                                     (gr.levels > 1 ? (size_t)residual_blocks(nt, c->lv[1].g.P) : 0)));
    LAMCHK(dalloc(&c->d_red, 1));
    LAMCHK(dalloc(&c->d_g, (size_t)P0));
    LAMCHK(dalloc(&c->d_cf, (size_t)P0 * nt));
    LAMCHK(dalloc(&c->d_Gpart, (size_t)c->max_parts * nt * nt));
    LAMCHK(dalloc(&c->d_G, (size_t)nt * nt));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_red), sizeof(double), hipHostMallocMapped) != hipSuccess)
        return LAM_ENOMEM;
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->h_red_dev), c->h_red, 0));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_norms), sizeof(double) * (c->solver.max_cycles + 3),
                      hipHostMallocMapped) != hipSuccess)
        return LAM_ENOMEM;
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->h_norms_dev), c->h_norms, 0));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_citers), sizeof(int) * (c->solver.max_cycles + 3),
                      hipHostMallocMapped) != hipSuccess)
        return LAM_ENOMEM;
    std::memset(c->h_citers, 0, sizeof(int) * (c->solver.max_cycles + 3));
    HIPCHK(hipHostGetDevicePointer(reinterpret_cast<void**>(&c->h_citers_dev), c->h_citers, 0));
    LAMCHK(dalloc(&c->d_ctl, 1));
    HIPCHK(hipMemsetAsync(c->d_ctl, 0, sizeof(CoarseCtl), c->st));
    c->coarse_launch = gr.nu_coarse;
    HIPCHK(hipEventCreateWithFlags(&c->ev_norm, hipEventDisableTiming));
    if (hipHostMalloc(reinterpret_cast<void**>(&c->h_G), sizeof(double2) * nt * nt) != hipSuccess)
        return LAM_ENOMEM;
    {
        // time factor records without field (forward, adjoint) for every step
        // length dt / 2^d a split may use, and the per-slab tables and staging
        // buffers for steps with a field
        const int TS = tf_record_stride(nt);
        c->TS = TS;
        const int nd = c->solver.max_split + 1;
        std::vector<double> h(2 * (size_t)nd * TS);
        c->h_tf0.resize(2 * nd);
        for (int d = 0; d < nd; ++d) {
            set_depth(c, d);
            for (int dir = 0; dir < 2; ++dir) {
                double* rec = h.data() + (2 * d + dir) * (size_t)TS;
                if (!make_record(c, nullptr, 0.0, dir, rec)) return LAM_EINVAL;
                c->h_tf0[2 * d + dir].assign(rec, rec + TS);
            }
        }
        set_depth(c, 0);
        std::vector<float> hf(h.begin(), h.end());
        LAMCHK(dalloc(&c->d_tf0, h.size()));
        LAMCHK(dalloc(&c->d_tf0f, hf.size()));
        HIPCHK(hipMemcpy(c->d_tf0, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c->d_tf0f, hf.data(), sizeof(float) * hf.size(), hipMemcpyHostToDevice));
        const size_t tb = tf_table_bytes(c);
        for (int dir = 0; dir < 2; ++dir) LAMCHK(dalloc(&c->d_tfs[dir], tb));
        for (auto& s : c->stage) {
            if (hipHostMalloc(reinterpret_cast<void**>(&s.h), tb) != hipSuccess) {
                s.h = nullptr;
                return LAM_ENOMEM;
            }
            HIPCHK(hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
        }
    }
    for (auto& L : c->lv) LAMCHK(factor_level(c, L));
    HIPCHK(hipStreamSynchronize(c->st));
    return LAM_OK;
}

// ---------------------------------------------------------------------------
// Steps, split in halves while their solves fail (solver max_split > 0).
// ---------------------------------------------------------------------------

// Statistics of the solves of one call: the work of every solve (including the
// abandoned ones), and for the accepted (sub-)steps the worst ratio of final to
// initial residual (resid0 / resid), the last step's, their count and the
// deepest halving.
struct Totals {
    lam_stats s{};
    double worst = -1.0;
    void work(const lam_stats& st) {
        s.cycles += st.cycles;
        s.coarse_sweeps += st.coarse_sweeps;
        s.coarse_unmet += st.coarse_unmet;
    }
    void accept(const lam_stats& st, int depth) {
        s.resid0_last = st.resid0;
        s.resid_last = st.resid;
        const double ratio = st.resid0 > 0.0 ? st.resid / st.resid0 : 0.0;
        if (ratio > worst) {
            worst = ratio;
            s.resid0 = st.resid0;
            s.resid = st.resid;
        }
        s.substeps += 1;
        s.split_depth = std::max(s.split_depth, depth);
    }
};

bool splittable(const lam_ctx* c, int rc, int depth) {
    return (rc == LAM_EDIVERGED || rc == LAM_ENOCONV) && depth < c->solver.max_split;
}

// The two buffers of halving depth d (allocated on first use).
int split_buffers(lam_ctx* c, int d, double2** mid, double2** gmid) {
    if ((int)c->d_split.size() <= d) c->d_split.resize(d + 1, nullptr);
    const size_t P = (size_t)c->lv[0].g.P;
    if (!c->d_split[d]) LAMCHK(dalloc(&c->d_split[d], 2 * P));
    *mid = c->d_split[d];
    *gmid = c->d_split[d] + P;
    return LAM_OK;
}

int forward_halves(lam_ctx* c, double t0, int depth, const double2* psi_in, double2* psi_out, Totals& tot);

// The forward step [t0, t0 + dt / 2^depth) from psi_in to psi_out.  A solve that
// fails while a further halving is allowed is replaced by the two halves.
// psi_in may be psi_out, or the finest level's constraint right-hand side
// (which holds the step's initial state and is not written by its solve).
int forward_split(lam_ctx* c, double t0, int depth, const double2* psi_in, double2* psi_out, Totals& tot) {
    set_depth(c, depth);
    LAMCHK(set_step(c, t0, 0));
    Level& L = c->lv[0];
    HIPCHK(launch_init_forward(c->nt, L.g.P, psi_in, L.d_c, L.d_lam, L.d_bs, c->st));
    c->adjoint = 0;
    c->have_state = 1;
    c->state_t0 = t0;
    c->state_depth = depth;
    lam_stats st{};
    const int rc = solve_loop(c, &st);
    tot.work(st);
    if (splittable(c, rc, depth)) return forward_halves(c, t0, depth + 1, psi_in, psi_out, tot);
    if (rc != LAM_OK && rc != LAM_ENOCONV) return rc;
    tot.accept(st, depth);
    HIPCHK(launch_end_eval(c->nt, L.g.P, L.d_c, psi_out, c->st));
    return rc;
}

// Two steps of length dt / 2^depth from t0 (the halves of a step of twice that).
int forward_halves(lam_ctx* c, double t0, int depth, const double2* psi_in, double2* psi_out, Totals& tot) {
    const int r1 = forward_split(c, t0, depth, psi_in, psi_out, tot);
    if (r1 != LAM_OK && r1 != LAM_ENOCONV) return r1;
    const int r2 = forward_split(c, t0 + std::ldexp(c->time.dt, -depth), depth, psi_out, psi_out, tot);
    return r2 != LAM_OK ? r2 : r1;
}

// The adjoint of the forward step [t0, t0 + dt / 2^depth) from psi_in (the
// forward solve is recomputed first, and decides whether the step splits, as
// it did going forward): g_in = the adjoint state at the step's start for
// g_out at its end, gradients accumulated.  A split step's adjoint runs
// through its halves in reverse, with the state between them recomputed.
int adjoint_gradients(lam_ctx* c, double t0, int depth, const double2* cf, const double2* g_out, double2* g_in,
                      double* dL_dv0, double* dL_dcoef, Totals& tot);

int adjoint_split(lam_ctx* c, double t0, int depth, const double2* psi_in, const double2* g_out, double2* g_in,
                  double* dL_dv0, double* dL_dcoef, Totals& tot) {
    set_depth(c, depth);
    LAMCHK(set_step(c, t0, 0));
    Level& L = c->lv[0];
    const int nt = c->nt;
    const size_t P = L.g.P;
    // 1. recompute the forward solution of this step from its checkpoint (the host
    //    builds the adjoint time factor records meanwhile)
    HIPCHK(launch_init_forward(nt, (int)P, psi_in, L.d_c, L.d_lam, L.d_bs, c->st));
    c->adjoint = 0;
    c->have_state = 1;
    c->state_t0 = t0;
    c->state_depth = depth;
    if (c->field_on) {
        c->prep_t = t0;
        c->prep_dir = 1;
    }
    int rc = solve_loop(c, nullptr);
    c->prep_t = NAN;
    if (splittable(c, rc, depth)) {
        double2 *mid, *gmid;
        LAMCHK(split_buffers(c, depth + 1, &mid, &gmid));
        Totals fwd;
        rc = forward_split(c, t0, depth + 1, psi_in, mid, fwd);
        if (rc != LAM_OK) return rc;
        const double th = t0 + std::ldexp(c->time.dt, -(depth + 1));
        LAMCHK(adjoint_split(c, th, depth + 1, mid, g_out, gmid, dL_dv0, dL_dcoef, tot));
        return adjoint_split(c, t0, depth + 1, psi_in, gmid, g_in, dL_dv0, dL_dcoef, tot);
    }
    if (rc != LAM_OK) return rc;
    // the adjoint solve overwrites the state: the forward solution moves aside
    HIPCHK(launch_copy_c2(L.d_c, c->d_cf, P * nt, c->st));
    return adjoint_gradients(c, t0, depth, c->d_cf, g_out, g_in, dL_dv0, dL_dcoef, tot);
}

// The adjoint solve of the step [t0, t0 + dt / 2^depth) and its gradients, for
// the converged forward coefficients cf of that step (device, P n_t, read only):
// g_in = the adjoint state at the step's start for g_out at its end, dL_dv0 and
// dL_dcoef accumulated.  The depth must already be set.
int adjoint_gradients(lam_ctx* c, double t0, int depth, const double2* cf, const double2* g_out, double2* g_in,
                      double* dL_dv0, double* dL_dcoef, Totals& tot) {
    Level& L = c->lv[0];
    const int nt = c->nt;
    const size_t P = L.g.P;
    c->have_state = 1;
    c->state_t0 = t0;
    c->state_depth = depth;
    // 2. adjoint solve K^H mu = E^H g_out from mu = 0
    LAMCHK(set_step(c, t0, 1));
    HIPCHK(launch_copy_c2(g_out, c->d_g, P, c->st));
    HIPCHK(launch_init_zero(nt, (int)P, L.d_c, L.d_lam, c->st));
    c->adjoint = 1;
    lam_stats st{};
    const int rc = solve_loop(c, &st);
    tot.work(st);
    if (rc != LAM_OK && rc != LAM_ENOCONV) return rc;
    tot.accept(st, depth);
    // 3. gradients
    int np = 0;
    const bool want_coef = dL_dcoef && !c->coef.empty() &&
                           (c->ham.pulse_kind == LAM_PULSE_FOURIER || c->ham.pulse_kind == LAM_PULSE_SIN2_FOURIER);
    HIPCHK(launch_gradients(nt, L.g, c->U, cf, L.d_c, dL_dv0, want_coef ? c->d_Gpart : nullptr, &np, c->st));
    HIPCHK(launch_copy_c2(L.d_lam, g_in, P, c->st));
    if (want_coef) {
        HIPCHK(launch_reduce_c2(c->d_Gpart, np, nt * nt, c->d_G, c->st));
        HIPCHK(hipMemcpyAsync(c->h_G, c->d_G, sizeof(double2) * nt * nt, hipMemcpyDeviceToHost, c->st));
    }
    HIPCHK(hipStreamSynchronize(c->st));
    if (want_coef) {
        double Wq[kMaxNT * kMaxNT];
        for (size_t q = 0; q < c->coef.size(); ++q) {
            time_matrix(c, t0, (int)q, Wq);
            double acc = 0.0;
            for (int m = 0; m < nt; ++m)
                for (int n = 0; n < nt; ++n) acc += Wq[m * nt + n] * c->h_G[m * nt + n].x;
            dL_dcoef[q] += 2.0 * acc;
        }
    }
    return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of lam_residual_action_noalloc: the per-workgroup
// partial sums of its norm reduction.  Each GPU the library runs on holds its
// own copy until the process ends; host code uses the address looked up per
// device below, never the array's name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) double scratch[LAM_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (looked up once per device).
int scratch_address(double** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return LAM_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return LAM_EHIP;
        g_scratch_ptr[dev] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[dev];
    return LAM_OK;
}

}  // namespace

extern "C" {

int lam_create(const lam_grid* grid, const lam_time* time, const lam_ham* ham, const lam_solver* solver,
               void* hip_stream, lam_ctx** out) {
    if (!out) return LAM_EINVAL;
    *out = nullptr;
    LAMCHK(validate(grid, time, ham, solver));
    lam_ctx* c = new (std::nothrow) lam_ctx();
    if (!c) return LAM_ENOMEM;
    c->grid = *grid;
    c->time = *time;
    c->ham = *ham;
    c->solver = *solver;
    c->st = static_cast<hipStream_t>(hip_stream);
    c->nt = time->n_t;
    c->L = grid->levels;
    c->coef.assign(ham->coef, ham->coef + ham->n_coef);
    c->ham.coef = nullptr;
    c->ham.v0 = nullptr;
    set_depth(c, 0);
    const int r = build(c, ham->v0);
    if (r != LAM_OK) {
        free_ctx(c);
        return r;
    }
    *out = c;
    return LAM_OK;
}

int lam_destroy(lam_ctx* ctx) {
    free_ctx(ctx);
    return LAM_OK;
}

int lam_set_pulse(lam_ctx* ctx, int n_coef, const double* coef) {
    if (!ctx || n_coef != (int)ctx->coef.size() || (n_coef > 0 && !coef)) return LAM_EINVAL;
    ctx->coef.assign(coef, coef + n_coef);
    // field matrices, time factor records and stored inverses must be rebuilt
    ctx->t0 = NAN;
    ctx->tf_t[0] = ctx->tf_t[1] = NAN;
    for (auto& s : ctx->stage) s.t = NAN;
    ctx->mf_t = NAN;
    if (ctx->have_state) {
        set_depth(ctx, ctx->state_depth);
        LAMCHK(set_step(ctx, ctx->state_t0, ctx->adjoint));
        set_depth(ctx, 0);
    }
    return LAM_OK;
}

int lam_set_potential(lam_ctx* ctx, const double* v0) {
    if (!ctx || !v0) return LAM_EINVAL;
    HIPCHK(hipMemcpyAsync(ctx->lv[0].d_v0, v0, sizeof(double) * ctx->lv[0].g.P, hipMemcpyDeviceToDevice, ctx->st));
    for (int l = 1; l < ctx->L; ++l)
        HIPCHK(launch_average_potential(ctx->lv[l - 1].g, ctx->lv[l].g, ctx->lv[l - 1].d_v0, ctx->lv[l].d_v0,
                                        ctx->st));
    for (auto& L : ctx->lv) LAMCHK(factor_level(ctx, L));
    if (ctx->have_state) {
        set_depth(ctx, ctx->state_depth);
        LAMCHK(set_step(ctx, ctx->state_t0, ctx->adjoint));
        set_depth(ctx, 0);
    }
    HIPCHK(hipStreamSynchronize(ctx->st));
    return LAM_OK;
}

int lam_residual_action(lam_ctx* ctx, double t0, const lam_c64* psi0, const lam_c64* c, const lam_c64* lam,
                        lam_c64* rho, lam_c64* sigma, double* norm) {
    if (!ctx || bad_ptr(psi0) || bad_ptr(c) || bad_ptr(lam)) return LAM_EINVAL;
    // the step's field matrix, without touching the step of the context's state
    double W[kMaxNT * kMaxNT];
    const int on = step_field(ctx, t0, W) ? 1 : 0;
    Level& L = ctx->lv[0];
    int np = 0;
    HIPCHK(launch_residual(ctx->nt, L.g, ctx->U, W, 0, on, reinterpret_cast<const double2*>(c),
                           reinterpret_cast<const double2*>(lam), L.d_v0, nullptr, nullptr,
                           reinterpret_cast<const double2*>(psi0), reinterpret_cast<double2*>(rho),
                           reinterpret_cast<double2*>(sigma), norm ? ctx->d_partial : nullptr, &np, ctx->st));
    if (norm) {
        HIPCHK(launch_reduce(ctx->d_partial, np, 1, ctx->h_red_dev, ctx->st));
        LAMCHK(wait_stream(ctx));
        *norm = ctx->h_red[0];
    }
    return LAM_OK;
}

int lam_residual_adjoint(lam_ctx* ctx, double t0, const lam_c64* g, const lam_c64* mu_c, const lam_c64* mu_lam,
                         lam_c64* rho, lam_c64* sigma, double* norm) {
    if (!ctx || bad_ptr(g) || bad_ptr(mu_c) || bad_ptr(mu_lam)) return LAM_EINVAL;
    double W[kMaxNT * kMaxNT];
    const int on = step_field(ctx, t0, W) ? 1 : 0;
    Level& L = ctx->lv[0];
    int np = 0;
    HIPCHK(launch_residual(ctx->nt, L.g, ctx->U, W, 1, on, reinterpret_cast<const double2*>(mu_c),
                           reinterpret_cast<const double2*>(mu_lam), L.d_v0, nullptr,
                           reinterpret_cast<const double2*>(g), nullptr, reinterpret_cast<double2*>(rho),
                           reinterpret_cast<double2*>(sigma), norm ? ctx->d_partial : nullptr, &np, ctx->st));
    if (norm) {
        HIPCHK(launch_reduce(ctx->d_partial, np, 1, ctx->h_red_dev, ctx->st));
        LAMCHK(wait_stream(ctx));
        *norm = ctx->h_red[0];
    }
    return LAM_OK;
}

int lam_set_state(lam_ctx* ctx, double t0, const lam_c64* psi0, const lam_c64* c, const lam_c64* lam) {
    if (!ctx || bad_ptr(psi0) || bad_ptr(c) || bad_ptr(lam)) return LAM_EINVAL;
    set_depth(ctx, 0);
    LAMCHK(set_step(ctx, t0, 0));
    Level& L = ctx->lv[0];
    const size_t P = L.g.P;
    HIPCHK(launch_copy_c2(reinterpret_cast<const double2*>(psi0), L.d_bs, P, ctx->st));
    HIPCHK(launch_copy_c2(reinterpret_cast<const double2*>(c), L.d_c, P * ctx->nt, ctx->st));
    HIPCHK(launch_copy_c2(reinterpret_cast<const double2*>(lam), L.d_lam, P, ctx->st));
    ctx->adjoint = 0;
    ctx->have_state = 1;
    ctx->state_t0 = t0;
    ctx->state_depth = 0;
    return LAM_OK;
}

int lam_set_adjoint_state(lam_ctx* ctx, double t0, const lam_c64* g, const lam_c64* mu_c, const lam_c64* mu_lam) {
    if (!ctx || bad_ptr(g) || bad_ptr(mu_c) || bad_ptr(mu_lam)) return LAM_EINVAL;
    set_depth(ctx, 0);
    LAMCHK(set_step(ctx, t0, 1));
    Level& L = ctx->lv[0];
    const size_t P = L.g.P;
    HIPCHK(launch_copy_c2(reinterpret_cast<const double2*>(g), ctx->d_g, P, ctx->st));
    HIPCHK(launch_copy_c2(reinterpret_cast<const double2*>(mu_c), L.d_c, P * ctx->nt, ctx->st));
    HIPCHK(launch_copy_c2(reinterpret_cast<const double2*>(mu_lam), L.d_lam, P, ctx->st));
    ctx->adjoint = 1;
    ctx->have_state = 1;
    ctx->state_t0 = t0;
    ctx->state_depth = 0;
    return LAM_OK;
}

int lam_get_state(lam_ctx* ctx, lam_c64* c, lam_c64* lam) {
    if (!ctx || bad_ptr(c) || bad_ptr(lam)) return LAM_EINVAL;
    if (!ctx->have_state) return LAM_ESTATE;
    Level& L = ctx->lv[0];
    const size_t P = L.g.P;
    HIPCHK(launch_copy_c2(L.d_c, reinterpret_cast<double2*>(c), P * ctx->nt, ctx->st));
    HIPCHK(launch_copy_c2(L.d_lam, reinterpret_cast<double2*>(lam), P, ctx->st));
    return LAM_OK;
}

int lam_relax_sweep(lam_ctx* ctx, int level, int colour) {
    if (!ctx || level < 0 || level >= ctx->L || (colour != 0 && colour != 1)) return LAM_EINVAL;
    if (!ctx->have_state) return LAM_ESTATE;
    if (level > 0) {
        // a coarse level relaxes its own correction problem; it needs a right-hand side
        // produced by a V-cycle, so only the finest level is addressable on its own
        return LAM_EINVAL;
    }
    // the step of the loaded state (a residual call may have looked at another one)
    set_depth(ctx, ctx->state_depth);
    LAMCHK(set_step(ctx, ctx->state_t0, ctx->adjoint));
    const int rc = sweep(ctx, level, colour);
    set_depth(ctx, 0);
    return rc;
}

int lam_vcycle(lam_ctx* ctx, double* norm) {
    if (!ctx) return LAM_EINVAL;
    if (!ctx->have_state) return LAM_ESTATE;
    set_depth(ctx, ctx->state_depth);
    LAMCHK(set_step(ctx, ctx->state_t0, ctx->adjoint));
    int rc = vcycle(ctx, 0);
    if (rc == LAM_OK && norm) rc = norm0(ctx, norm);
    set_depth(ctx, 0);
    return rc;
}

int lam_solve_step(lam_ctx* ctx, double t0, const lam_c64* psi_in, lam_c64* psi_out, lam_stats* stats) {
    if (!ctx || bad_ptr(psi_in) || bad_ptr(psi_out)) return LAM_EINVAL;
    const auto t_a = std::chrono::steady_clock::now();
    ctx->t_factor_ms = 0.0;
    const int sw0 = ctx->sweeps_fine;
    Totals tot;
    const int rc = forward_split(ctx, t0, 0, reinterpret_cast<const double2*>(psi_in),
                                 reinterpret_cast<double2*>(psi_out), tot);
    set_depth(ctx, 0);
    if (rc != LAM_OK && rc != LAM_ENOCONV) return rc;
    LAMCHK(wait_stream(ctx));
    if (stats) {
        *stats = tot.s;
        stats->sweeps_fine = ctx->sweeps_fine - sw0;
        stats->t_factor_ms = ctx->t_factor_ms;
        stats->t_solve_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_a).count();
    }
    return rc;
}

int lam_propagate(lam_ctx* ctx, double t0, int n_steps, const lam_c64* psi_in, lam_c64* psi_out,
                  lam_stats* stats) {
    if (!ctx || bad_ptr(psi_in) || bad_ptr(psi_out)) return LAM_EINVAL;
    if (n_steps < 0) return LAM_EINVAL;
    const auto t_a = std::chrono::steady_clock::now();
    ctx->t_factor_ms = 0.0;
    const int sw0 = ctx->sweeps_fine;
    Level& L = ctx->lv[0];
    Totals tot;
    int rc = LAM_OK;
    const lam_c64* src = psi_in;
    double2* out = reinterpret_cast<double2*>(psi_out);
    int n0_slot = -1;  // >= 0: this step's initial state is in place and its N0 queued into that slot
    for (int k = 0; k < n_steps; ++k) {
        const double tk = t0 + k * ctx->time.dt;
        set_depth(ctx, 0);
        LAMCHK(set_step(ctx, tk, 0));
        if (n0_slot < 0)
            HIPCHK(launch_init_forward(ctx->nt, L.g.P, reinterpret_cast<const double2*>(src), L.d_c, L.d_lam,
                                       L.d_bs, ctx->st));
        ctx->adjoint = 0;
        ctx->have_state = 1;
        ctx->state_t0 = tk;
        ctx->state_depth = 0;
        // The next step's start (its initial state and N0, with its field) is
        // queued ahead of each wait for this step's norms, and while the GPU works
        // the host builds the next step's time factor records.
        double Wn[kMaxNT * kMaxNT];
        const double tn = t0 + (k + 1) * ctx->time.dt;
        const bool has_next = k + 1 < n_steps;
        const bool next_field = has_next && step_field(ctx, tn, Wn);
        if (next_field) {
            ctx->prep_t = tn;
            ctx->prep_dir = 0;
        }
        // (the step-ahead start computes the unrefined N0: not with the adaptive tree)
        const bool ahead = has_next && !ctx->refined && alloc_next(ctx);
        const int next_slot = ctx->solver.max_cycles + 1 + (k & 1);
        bool ready = false;
        lam_stats st{};
        rc = solve_loop(ctx, &st, n0_slot, ahead ? out : nullptr, next_slot, &ready, next_field ? Wn : nullptr);
        ctx->prep_t = NAN;
        tot.work(st);
        n0_slot = -1;
        if (splittable(ctx, rc, 0)) {
            // the step again as two halves, from its initial state (the finest
            // level's constraint right-hand side: the failed solve left it intact)
            rc = forward_halves(ctx, tk, 1, L.d_bs, out, tot);
            set_depth(ctx, 0);
            if (rc != LAM_OK && rc != LAM_ENOCONV) return rc;
        } else {
            if (rc != LAM_OK && rc != LAM_ENOCONV) return rc;
            tot.accept(st, 0);
            if (ready) {
                // psi_out holds this step's end state; the next step starts from the spare buffers
                std::swap(L.d_c, ctx->d_c_next);
                std::swap(L.d_lam, ctx->d_lam_next);
                std::swap(L.d_bs, ctx->d_bs_next);
                n0_slot = next_slot;
            } else {
                HIPCHK(launch_end_eval(ctx->nt, L.g.P, L.d_c, out, ctx->st));
            }
        }
        src = psi_out;
        if (rc != LAM_OK) break;
    }
    LAMCHK(wait_stream(ctx));
    if (stats) {
        *stats = tot.s;
        stats->sweeps_fine = ctx->sweeps_fine - sw0;
        stats->t_factor_ms = ctx->t_factor_ms;
        stats->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_a).count();
    }
    return rc;
}

int lam_adjoint_step(lam_ctx* ctx, double t0, const lam_c64* psi_in, const lam_c64* g_out, lam_c64* g_in,
                     double* dL_dv0, double* dL_dcoef, lam_stats* stats) {
    if (!ctx || bad_ptr(psi_in) || bad_ptr(g_out) || bad_ptr(g_in) || bad_ptr(dL_dv0)) return LAM_EINVAL;
    const auto t_a = std::chrono::steady_clock::now();
    ctx->t_factor_ms = 0.0;
    const int sw0 = ctx->sweeps_fine;
    Totals tot;
    // the adjoint step (forward recomputation included) solves the unrefined step
    ctx->refine_off = true;
    const int rc = adjoint_split(ctx, t0, 0, reinterpret_cast<const double2*>(psi_in),
                                 reinterpret_cast<const double2*>(g_out), reinterpret_cast<double2*>(g_in), dL_dv0,
                                 dL_dcoef, tot);
    ctx->refine_off = false;
    set_depth(ctx, 0);
    if (rc != LAM_OK && rc != LAM_ENOCONV) return rc;
    if (stats) {
        *stats = tot.s;
        stats->sweeps_fine = ctx->sweeps_fine - sw0;
        stats->t_factor_ms = ctx->t_factor_ms;
        stats->t_solve_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_a).count();
    }
    return rc;
}

int lam_adjoint_step_stored(lam_ctx* ctx, double t0, const lam_c64* c_fwd, const lam_c64* g_out, lam_c64* g_in,
                            double* dL_dv0, double* dL_dcoef, lam_stats* stats) {
    if (!ctx || bad_ptr(c_fwd) || bad_ptr(g_out) || bad_ptr(g_in) || bad_ptr(dL_dv0)) return LAM_EINVAL;
    const auto t_a = std::chrono::steady_clock::now();
    ctx->t_factor_ms = 0.0;
    const int sw0 = ctx->sweeps_fine;
    Totals tot;
    ctx->refine_off = true;
    set_depth(ctx, 0);
    const int rc = adjoint_gradients(ctx, t0, 0, reinterpret_cast<const double2*>(c_fwd),
                                     reinterpret_cast<const double2*>(g_out), reinterpret_cast<double2*>(g_in), dL_dv0,
                                     dL_dcoef, tot);
    ctx->refine_off = false;
    if (rc != LAM_OK && rc != LAM_ENOCONV) return rc;
    if (stats) {
        *stats = tot.s;
        stats->sweeps_fine = ctx->sweeps_fine - sw0;
        stats->t_factor_ms = ctx->t_factor_ms;
        stats->t_solve_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_a).count();
    }
    return rc;
}

int lam_set_refinement(lam_ctx* ctx, const unsigned char* active) {
    if (!ctx) return LAM_EINVAL;
    if (ctx->L < 2 || ctx->grid.coarse_op != LAM_COARSE_GALERKIN) return LAM_EINVAL;
    Level& L = ctx->lv[0];
    if (!active) {
        ctx->refined = false;
        return LAM_OK;
    }
    const LevelGeom& g = L.g;
    std::vector<int> col[2];
    std::vector<unsigned char> mask(L.nblocks);
    for (int b = 0; b < L.nblocks; ++b) {
        int bc[3] = {0, 0, 0}, t = b;
        for (int a = g.dim - 1; a >= 0; --a) {
            bc[a] = t % g.nblk[a];
            t /= g.nblk[a];
        }
        mask[b] = active[b] ? 1 : 0;
        if (active[b]) col[(bc[0] + bc[1] + bc[2]) & 1].push_back(b);
    }
    // the previous lists may still be read by queued sweeps
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (!ctx->d_bmask) LAMCHK(dalloc(&ctx->d_bmask, (size_t)L.nblocks));
    HIPCHK(hipMemcpy(ctx->d_bmask, mask.data(), mask.size(), hipMemcpyHostToDevice));
    for (int k = 0; k < 2; ++k) {
        if (!ctx->d_act[k]) LAMCHK(dalloc(&ctx->d_act[k], (size_t)std::max(1, L.ncol[k])));
        ctx->nact[k] = (int)col[k].size();
        if (!col[k].empty())
            HIPCHK(hipMemcpy(ctx->d_act[k], col[k].data(), sizeof(int) * col[k].size(), hipMemcpyHostToDevice));
    }
    ctx->refined = true;
    return LAM_OK;
}

int lam_block_detail(lam_ctx* ctx, const lam_c64* psi, double* detail) {
    if (!ctx || bad_ptr(psi) || bad_ptr(detail)) return LAM_EINVAL;
    Level& L = ctx->lv[0];
    double* d = nullptr;
    LAMCHK(dalloc(&d, (size_t)L.nblocks));
    hipError_t e = launch_block_detail(L.g, reinterpret_cast<const double2*>(psi), d, ctx->st);
    if (e == hipSuccess) e = hipMemcpyAsync(detail, d, sizeof(double) * L.nblocks, hipMemcpyDeviceToHost, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    (void)hipFree(d);
    return e == hipSuccess ? LAM_OK : LAM_EHIP;
}

int lam_restrict(lam_ctx* ctx, int level, const lam_c64* rho_f, const lam_c64* sigma_f, lam_c64* rho_c,
                 lam_c64* sigma_c) {
    if (!ctx || level < 0 || level + 1 >= ctx->L) return LAM_EINVAL;
    if (bad_ptr(rho_f) || bad_ptr(sigma_f) || bad_ptr(rho_c) || bad_ptr(sigma_c)) return LAM_EINVAL;
    HIPCHK(launch_restrict(ctx->nt, ctx->lv[level].g, ctx->lv[level + 1].g, reinterpret_cast<const double2*>(rho_f),
                           reinterpret_cast<const double2*>(sigma_f), reinterpret_cast<double2*>(rho_c),
                           reinterpret_cast<double2*>(sigma_c), nullptr, nullptr, ctx->st));
    return LAM_OK;
}

int lam_prolong_add(lam_ctx* ctx, int level, const lam_c64* c_c, const lam_c64* lam_c, lam_c64* c_f,
                    lam_c64* lam_f) {
    if (!ctx || level < 0 || level + 1 >= ctx->L) return LAM_EINVAL;
    if (bad_ptr(c_c) || bad_ptr(lam_c) || bad_ptr(c_f) || bad_ptr(lam_f)) return LAM_EINVAL;
    HIPCHK(launch_prolong(ctx->nt, ctx->lv[level].g, ctx->lv[level + 1].g, ctx->grid.interp,
                          reinterpret_cast<const double2*>(c_c), reinterpret_cast<const double2*>(lam_c),
                          reinterpret_cast<double2*>(c_f), reinterpret_cast<double2*>(lam_f), ctx->st));
    return LAM_OK;
}

int lam_level_shape(const lam_ctx* ctx, int level, int* n) {
    if (!ctx || !n || level < 0 || level >= ctx->L) return LAM_EINVAL;
    for (int a = 0; a < 3; ++a) n[a] = a < ctx->grid.dim ? ctx->lv[level].g.n[a] : 1;
    return LAM_OK;
}

int lam_block_factor(const lam_ctx* ctx, int level, int block, double* vecs, double* vals) {
    if (!ctx || !vecs || !vals || level < 0 || level >= ctx->L) return LAM_EINVAL;
    const Level& L = ctx->lv[level];
    if (block < 0 || block >= L.nblocks) return LAM_EINVAL;
    const size_t B = L.g.bpts;
    HIPCHK(hipStreamSynchronize(ctx->st));
    HIPCHK(hipMemcpy(vecs, L.d_V + block * B * B, sizeof(double) * B * B, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(vals, L.d_e + block * B, sizeof(double) * B, hipMemcpyDeviceToHost));
    return LAM_OK;
}

int lam_residual_action_noalloc(const lam_grid* grid, const lam_time* time, const lam_ham* ham, double t0,
                                const lam_c64* psi0, const lam_c64* c, const lam_c64* lam, lam_c64* rho,
                                lam_c64* sigma, double* norm, void* hip_stream) {
    const lam_solver any_solver{LAM_FP64, 0.0, 0, -1, LAM_TF_SHARED, 0.0};
    LAMCHK(validate(grid, time, ham, &any_solver));
    if (bad_ptr(psi0) || bad_ptr(c) || bad_ptr(lam)) return LAM_EINVAL;
    const int nt = time->n_t;
    const LevelGeom g = level_geom(*grid, *ham, 0);
    double U[kMaxNT], W[kMaxNT * kMaxNT];
    for (int m = 0; m < nt; ++m) U[m] = time->dt / (2.0 * m + 1.0);
    time_matrix(*ham, ham->coef, ham->n_coef, nt, time->dt, t0, -1, W);
    const int on = any_nonzero(W, nt * nt) ? 1 : 0;
    double* partial = nullptr;
    if (norm) {
        if ((size_t)residual_blocks(nt, g.P) > LAM_NOALLOC_SCRATCH_BYTES / sizeof(double)) return LAM_ETOOBIG;
        LAMCHK(scratch_address(&partial));
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    int np = 0;
    HIPCHK(launch_residual(nt, g, U, W, 0, on, reinterpret_cast<const double2*>(c),
                           reinterpret_cast<const double2*>(lam), ham->v0, nullptr, nullptr,
                           reinterpret_cast<const double2*>(psi0), reinterpret_cast<double2*>(rho),
                           reinterpret_cast<double2*>(sigma), partial, &np, st));
    if (norm) HIPCHK(launch_reduce(partial, np, 1, norm, st));
    return LAM_OK;
}

int lam_pass_stats(lam_ctx* ctx, int level, long long* hist) {
    if (!ctx || !hist || level < 0 || level >= ctx->L) return LAM_EINVAL;
    const Level& L = ctx->lv[level];
    std::vector<unsigned char> h((size_t)L.nblocks);
    HIPCHK(hipStreamSynchronize(ctx->st));
    HIPCHK(hipMemcpy(h.data(), L.d_passes, h.size(), hipMemcpyDeviceToHost));
    for (int k = 0; k < LAM_MAX_INNER + 2; ++k) hist[k] = 0;
    for (const unsigned char v : h) {
        hist[std::min(v & 0x7f, LAM_MAX_INNER)]++;
        if (v & 0x80) hist[LAM_MAX_INNER + 1]++;
    }
    return LAM_OK;
}

int lam_profile(lam_ctx* ctx, int enable) {
    if (!ctx) return LAM_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->st));
    if (enable < 0) return LAM_EINVAL;
    ctx->prof = enable;
    ctx->prof_count = 0;
    if (enable) ctx->nev = 0;
    return LAM_OK;
}

int lam_profile_read(lam_ctx* ctx, int* launches, double* total_ms) {
    if (!ctx || !launches || !total_ms) return LAM_EINVAL;
    HIPCHK(hipStreamSynchronize(ctx->st));
    double tot = 0.0;
    for (int k = 0; k + 1 < ctx->nev; k += 2) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, ctx->ev[k], ctx->ev[k + 1]));
        tot += ms;
    }
    *launches = ctx->nev / 2;
    *total_ms = tot;
    return LAM_OK;
}

const char* lam_strerror(int code) {
    switch (code) {
        case LAM_OK: return "ok";
        case LAM_EINVAL: return "invalid argument";
        case LAM_ENOMEM: return "device allocation failed";
        case LAM_EHIP: return "HIP runtime error";
        case LAM_ENOCONV: return "tolerance not reached within max_cycles";
        case LAM_EDIVERGED: return "residual norm diverged";
        case LAM_ESTATE: return "no state loaded";
        case LAM_ETOOBIG: return "input larger than the fixed scratch of a no-allocation call";
        default: return "unknown error";
    }
}

}  // extern "C"
