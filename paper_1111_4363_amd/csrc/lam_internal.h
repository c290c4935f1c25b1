// Internal declarations shared by the kernels and the host side of liblam.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "lam.h"

namespace lam {

constexpr int kMaxNT = LAM_MAX_NT;
constexpr int kMaxB = LAM_MAX_BLOCK;
constexpr int kThreads = 256;
constexpr int kSweepThreads = 512;   // the colour sweep: 8 waves per block, one lane per (point, component)
constexpr int kPairThreads = 256;    // its FP32 shared-factor form: 4 waves per block, two components per lane
constexpr int kLdsPad = kMaxB + 1;   // row stride of per-block matrices in LDS

// Geometry of one level, passed by value to kernels.
struct LevelGeom {
    int dim;
    int n[3];        // points per axis (unused axes = 1)
    int P;           // total points
    double h;
    int periodic;
    int fax;         // dipole axis
    double kin;      // 1/(2 m h^2): T = -kin * (sum of neighbours - 2 d u)
    int bdim[3];     // block points per axis (unused axes = 1)
    int nblk[3];     // blocks per axis
    int bpts;        // points per block
    double rn[3];    // 1 / n[a], for division-free index arithmetic
    double rnb[3];   // 1 / nblk[a]
    float rbd[3];    // 1 / bdim[a]
    float rbp;       // 1 / bpts
};

// Time operators of one step: diagonal of U and the field matrix W (symmetric).
template <int NT>
struct TimeOps {
    double U[NT];
    double W[NT * NT];
};

struct SweepArgs {
    // first: what a workgroup needs to find its block (read together at entry)
    int colour;               // the colour relaxed (parity of the sum of block coordinates)
    int arith_blocks;         // 1: the block grid's last axis has an even count, and the
                              //    colour's blocks are enumerated arithmetically (no table)
    int half_last;            // half the block count of the last axis (arithmetic enumeration)
    int pad_;
    LevelGeom g;
    const int* blocks;        // block ids of the colour being relaxed
    double2* c;               // [P][NT]
    double2* lam;             // [P]
    const double* v0;         // [P]
    const double2* bc;        // stationarity right-hand side [P][NT], may be null
    const double2* bg;        // or: the same value on every row (j, n): bg[j]; may be null
    const double2* bs;        // constraint right-hand side [P], may be null (= 0)
    const void* V;            // [nblocks][bpts][bpts] eigenvectors (double or float)
    const void* Minv;         // [nblocks][NT+1][NT+1][bpts] mode inverses (double2 or float2), or null:
    const void* tf;           // time factor records of this level and direction (double or float),
                              // one per slab of blocks along the field axis (layout below)
    int tf_stride;            // reals from one slab's record to the next; 0: one record for all
    int pad2_;
    const double* e;          // [nblocks][bpts] eigenvalues of the block operators
    unsigned char* passes;    // [nblocks] inner passes of each block's last solve (bit 7: its
                              // local system was left unsolved); may be null
    const int* skip;          // when non-null and nonzero at launch, the launch does nothing
    int adjoint;
    int n_inner;
    int field_on;             // W (the field's time matrix) is nonzero this step
    double inner_tol2;        // inner passes stop once the block's residual norm fell by
                              // this factor squared
    double wbound2;           // square of an upper bound of the 2-norm of W (its largest
                              // absolute row sum; W is symmetric), 0 without a field
};

// Control of the iterated coarsest-level solve (device memory): the norm N of
// the coarsest residual when the solve started and after the latest sweep,
// whether the reduction is reached (the remaining launches of the solve then
// do nothing) and the number of full sweeps that ran.
struct CoarseCtl {
    double n0;
    double n;
    int done;
    int iters;
};

// A time factor record (reals of the factor's precision): the real forms
// (2 n_t x 2 n_t, acting on interleaved re/im) of E1 and E3, then lam (n_t
// complex), then the dipole coordinate zf the factor was built for, then one
// pad entry.  See time_factor() in lam_api.hip.
constexpr int tf_record_reals(int nt) { return 8 * nt * nt + 2 * nt; }   // E1, E3, lam
constexpr int tf_record_stride(int nt) { return tf_record_reals(nt) + 2; } // + zf + pad

constexpr int kMaxInner = 32;   // most inner passes of one subvolume solve

// Workgroups (and norm partials) of a residual launch over P points.
inline int residual_blocks(int nt, int P) {
    const int pw = kThreads / nt;
    return (P + pw - 1) / pw;
}

// ---- launchers (lam_kernels.hip) -------------------------------------------
// All return hipSuccess or the launch error.

// skip (may be null): when it points to a nonzero value at launch, the launch does nothing.
hipError_t launch_residual(int nt, const LevelGeom& g, const double* U, const double* W, int adjoint,
                           int field_on, const double2* c, const double2* lam, const double* v0, const double2* bc,
                           const double2* bg, const double2* bs, double2* rc, double2* rs, double* partial,
                           int* nparts, hipStream_t st, const int* skip = nullptr,
                           const unsigned char* bmask = nullptr);
// bmask (may be null): one flag per subvolume of g; the norm partials count only
// the rows of flagged subvolumes (the residual fields are written in full).

// Partials of sum_j sum_m U_m |rho_jm|^2 + |sigma_j|^2 over P points (as many as
// residual_blocks(nt, P)).
hipError_t launch_rhs_norm(int nt, int P, const double* U, const double2* rho, const double2* sig, double* partial,
                           int* nparts, hipStream_t st);

// Haar detail energy of psi per subvolume of g (blocks of at most 64 points).
hipError_t launch_block_detail(const LevelGeom& g, const double2* psi, double* out, hipStream_t st);

hipError_t launch_reduce(const double* partial, int nparts, int width, double* out, hipStream_t st);

// Sum of the partials into the coarsest-solve control: start = 1 opens a solve
// (n0 = n = sum, done = (sum == 0), iters = 0); start = 0 closes one full sweep
// unless the solve is already done (iters + 1, n = sum, done = n <= thr2 n0).
// iters_out (may be null, e.g. mapped host memory) receives iters and, in bit
// 30, whether the reduction was reached.
hipError_t launch_reduce_ctl(const double* partial, int nparts, CoarseCtl* ctl, int start, double thr2,
                             int* iters_out, hipStream_t st);

hipError_t launch_residual_restrict(int nt, const LevelGeom& fine, const LevelGeom& coarse, const double* U,
                                    const double* W, int adjoint, int field_on, const double2* c,
                                    const double2* lam, const double* v0, const double2* bc, const double2* bg,
                                    const double2* bs, double2* bcc, double2* bsc, double2* zero_c,
                                    double2* zero_l, hipStream_t st);
hipError_t launch_restrict(int nt, const LevelGeom& fine, const LevelGeom& coarse, const double2* rcf,
                           const double2* rsf, double2* bcc, double2* bsc, double2* zero_c,
                           double2* zero_l, hipStream_t st);

hipError_t launch_prolong(int nt, const LevelGeom& fine, const LevelGeom& coarse, int interp,
                          const double2* cc, const double2* lc, double2* cf, double2* lf,
                          hipStream_t st);

hipError_t launch_average_potential(const LevelGeom& fine, const LevelGeom& coarse, const double* vf,
                                    double* vc, hipStream_t st);

hipError_t launch_block_eig(const LevelGeom& g, const double* v0, double* V, double* e, float* Vf,
                            hipStream_t st);

// Per-mode inverses of the full time systems of every block of a level, with
// the field's time matrix W taken at the zf of each block's slab record in tf
// (FP64 records, stride tf_stride; tf null or W null: no field).
hipError_t launch_mode_factor(int nt, const LevelGeom& g, const double* U, const double* W, const double* e,
                              const double* tf, int tf_stride, double2* Minv, float2* Minvf, hipStream_t st);

hipError_t launch_sweep(int nt, int mixed, const SweepArgs& a, const double* U, const double* W,
                        int nblocks_colour, hipStream_t st);

hipError_t launch_init_forward(int nt, int P, const double2* psi, double2* c, double2* lam, double2* bs,
                               hipStream_t st);

hipError_t launch_init_zero(int nt, int P, double2* c, double2* lam, hipStream_t st);

hipError_t launch_end_eval(int nt, int P, const double2* c, double2* psi, hipStream_t st);

// psi = end state of c; (cn, lamn, bsn) = the next step's initial state from
// psi; partial = per-workgroup partials of that state's N0 (U, W: the time
// operators of the next step, W null without field; *nparts of them,
// residual_blocks(nt, P)).
hipError_t launch_advance(int nt, const LevelGeom& g, const double* U, const double* W, const double2* c,
                          const double* v0, double2* psi, double2* cn, double2* lamn, double2* bsn,
                          double* partial, int* nparts, hipStream_t st);

hipError_t launch_copy_c2(const double2* src, double2* dst, size_t n, hipStream_t st);

hipError_t launch_gradients(int nt, const LevelGeom& g, const double* U, const double2* cfwd,
                            const double2* mu, double* dv0, double2* Gpart, int* nparts,
                            hipStream_t st);

hipError_t launch_reduce_c2(const double2* partial, int nparts, int width, double2* out,
                            hipStream_t st);

}  // namespace lam
