// HIP kernels of liblam for gfx950 (CDNA4, wave64).
//
// Layout in HBM: per grid point, n_t consecutive complex FP64 coefficients
// c[j][n] (interleaved re/im), one complex multiplier lam[j], one real V0[j].
// Grid points are in C order over the axes.  Per subvolume ("block"): the
// eigenvectors of its real symmetric spatial operator [point][mode] (FP64, and
// an FP32 copy for the mixed path) and its eigenvalues.  Time factors (the
// eigenbasis form of the n_t x n_t time system left once each point's
// continuity row has eliminated dc_0): one record shared by all blocks for a
// step without field, and with a field one per slab of blocks along the field
// axis, built with the field's time matrix at the slab's centre coordinate.
// Optionally, per mode, the inverse of the full (n_t+1) x (n_t+1) system,
// stored [block][row][col][mode] so that one wave reads 64 modes of one entry
// as a contiguous segment.

#include "lam_internal.h"

namespace lam {
namespace {

// ---------------------------------------------------------------------------
// small complex helpers (T = float or double)
// ---------------------------------------------------------------------------
template <typename T>
struct cx {
    T r, i;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // conj(a) * b
    return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
template <typename T>
__device__ __forceinline__ cx<T> rmul(T s, cx<T> a) { return {s * a.r, s * a.i}; }

// ---------------------------------------------------------------------------
// 16x16x4 matrix-core tiles (one wave).  Operand layout (checked on gfx950):
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k; the 16x16 result has
// column j = lane % 16 and, per result slot r, row
//   FP64: i = lane/16 + 4r          FP32: i = 4(lane/16) + r.
// ---------------------------------------------------------------------------
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// One 16 x 16 output tile per wave of out[m][c] = sum_p Op(m, p) in[p][c]
// (m, p < b, c < ncol <= 32; rows of in LD apart), with Op(m, p) = Vs[p][m]
// (TRANS: into the block eigenbasis) or Vs[m][p] (back to points).  Wave w owns rows 16 (w % 4) ..
// and columns 16 (w / 4) ..; every operand load is unconditional (clamped
// address times a 0/1 factor) so successive K steps stay in flight.
template <typename T, bool TRANS, int NCOL, int LD>
__device__ __forceinline__ typename Mfma<T>::acc_t tile_gemm(const T* __restrict__ Vs, const T* __restrict__ in,
                                                             int b, int lane, int wave) {
    typename Mfma<T>::acc_t acc;
    for (int r = 0; r < 4; ++r) acc[r] = (T)0;
    const int mt = wave & 3, nt = wave >> 2;
    if (16 * mt >= b || 16 * nt >= NCOL) return acc;
    const int i = lane & 15, kq = lane >> 4;
    const int m = 16 * mt + i, col = 16 * nt + i;
    // columns past NCOL only feed result columns that are never stored: read column NCOL-1
    const int cc = col < NCOL ? col : NCOL - 1;
    if (b == kMaxB) {
        // full block: every operand in range.  Step s takes K index p = 16 kq + s
        // from lane group kq, so the four groups of a step read V rows (or columns)
        // 16 apart: distinct LDS banks with the padded row stride.  Two halves of
        // eight steps, each half's loads issued together, offsets folded into the
        // LDS instructions.
#pragma unroll 1
        for (int sh = 0; sh < kMaxB / 4; sh += kMaxB / 8) {
            const int p0 = 16 * kq + sh;
            const T* va = TRANS ? Vs + p0 * kLdsPad + m : Vs + m * kLdsPad + p0;
            const T* vb = in + p0 * LD + cc;
#pragma unroll
            for (int s = 0; s < kMaxB / 8; ++s) {
                const T av = TRANS ? va[s * kLdsPad] : va[s];
                acc = Mfma<T>::step(av, vb[s * LD], acc);
            }
        }
        return acc;
    }
    const T fm = m < b ? (T)1 : (T)0;
    const int mc = m < b ? m : b - 1;
    // K in groups of 16 (four MFMA steps): the group's loads are issued together
    for (int kb = 0; kb < kMaxB; kb += 16) {
        if (kb >= b) break;
        T av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = kb + 4 * u + kq;
            const T fp = p < b ? (T)1 : (T)0;
            const int pc = p < b ? p : b - 1;
            av[u] = (TRANS ? Vs[pc * kLdsPad + mc] : Vs[mc * kLdsPad + pc]) * (fm * fp);
            bv[u] = in[pc * LD + cc];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = Mfma<T>::step(av[u], bv[u], acc);
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ void tile_store(T* __restrict__ out, int b, int ncol, int ld, int lane, int wave,
                                           const typename Mfma<T>::acc_t& acc) {
    const int mt = wave & 3, nt = wave >> 2;
    if (16 * mt >= b || 16 * nt >= ncol) return;
    for (int r = 0; r < 4; ++r) {
        const int m = 16 * mt + Mfma<T>::row(lane, r);
        const int col = 16 * nt + (lane & 15);
        if (m < b && col < ncol) out[m * ld + col] = acc[r];
    }
}

__device__ __forceinline__ double2 add2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 sub2(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 scl2(double s, double2 a) { return make_double2(s * a.x, s * a.y); }

// ---------------------------------------------------------------------------
// grid indexing.  Coordinates are three scalars; axes beyond the grid's rank
// have extent 1 (n, bdim, nblk), so the three-axis C-order formulas hold for
// 1D, 2D and 3D alike and no loop is bounded by the rank.
// ---------------------------------------------------------------------------
struct I3 {
    int x, y, z;
};

__device__ __forceinline__ int comp(const I3& v, int ax) { return ax == 0 ? v.x : (ax == 1 ? v.y : v.z); }

__device__ __forceinline__ I3 with_comp(I3 v, int ax, int val) {
    if (ax == 0) v.x = val;
    else if (ax == 1) v.y = val;
    else v.z = val;
    return v;
}

// Quotients without integer division: floor(j / n) as (j + 1/2) times the
// rounded reciprocal 1/n, truncated.  (j + 1/2)/n lies at least 1/(2n) from an
// integer and the two roundings move it by at most (j + 1/2)/n * 2 eps, so the
// quotient is exact when (j + 1/2) * 2 eps < 1/2: for 0 <= j < 2^31 in FP64
// (qdiv) and for 0 <= j < 2^21 in FP32 (qdiv_small), for any n >= 1.
__device__ __forceinline__ int qdiv(int j, double rn) { return (int)(((double)j + 0.5) * rn); }
__device__ __forceinline__ int qdiv_small(int j, float rn) { return (int)(((float)j + 0.5f) * rn); }

__device__ __forceinline__ I3 point_coords(const LevelGeom& g, int j) {
    I3 i;
    const int t = qdiv(j, g.rn[2]);
    i.z = j - t * g.n[2];
    i.x = qdiv(t, g.rn[1]);
    i.y = t - i.x * g.n[1];
    return i;
}

__device__ __forceinline__ int point_index(const LevelGeom& g, const I3& i) {
    return (i.x * g.n[1] + i.y) * g.n[2] + i.z;
}

// Neighbour of point i along axis ax in direction d: global index, or -1
// outside a Dirichlet grid.  *gi receives the (wrapped) coordinates.
__device__ __forceinline__ int neighbour(const LevelGeom& g, const I3& i, int ax, int d, I3* gi) {
    const int na = g.n[ax];
    int v = comp(i, ax) + d;
    if (v < 0 || v >= na) {
        if (!g.periodic) return -1;
        v += v < 0 ? na : -na;
    }
    *gi = with_comp(i, ax, v);
    return point_index(g, *gi);
}

// The same neighbour found from the point's own index and the axis stride, as
// selects (no branches): j +- stride inside the grid, the opposite end of the
// axis across a periodic boundary, -1 outside a Dirichlet grid.  AX and D are
// compile-time, so the stride and the wrap offset are uniform values.
template <int AX, int D>
__device__ __forceinline__ int neighbour_of(const LevelGeom& g, const I3& i, int j) {
    const int na = g.n[AX];
    const int st = AX == 2 ? 1 : (AX == 1 ? g.n[2] : g.n[1] * g.n[2]);
    const int v = comp(i, AX) + D;
    const int wrap = g.periodic ? j - D * (na - 1) * st : -1;
    return (unsigned)v < (unsigned)na ? j + D * st : wrap;
}

__device__ __forceinline__ double zcoord(const LevelGeom& g, const I3& i) {
    return (comp(i, g.fax) - 0.5 * (g.n[g.fax] - 1)) * g.h;
}

// Block bookkeeping: block id -> block coordinates; local index -> local coords.
__device__ __forceinline__ I3 block_coords(const LevelGeom& g, int blk) {
    I3 b;
    const int t = qdiv(blk, g.rnb[2]);
    b.z = blk - t * g.nblk[2];
    b.x = qdiv(t, g.rnb[1]);
    b.y = t - b.x * g.nblk[1];
    return b;
}

__device__ __forceinline__ I3 local_coords(const LevelGeom& g, int l) {
    I3 c;
    const int t = qdiv_small(l, g.rbd[2]);
    c.z = l - t * g.bdim[2];
    c.x = qdiv_small(t, g.rbd[1]);
    c.y = t - c.x * g.bdim[1];
    return c;
}

__device__ __forceinline__ int local_index(const LevelGeom& g, const I3& lc) {
    return (lc.x * g.bdim[1] + lc.y) * g.bdim[2] + lc.z;
}

__device__ __forceinline__ I3 global_of_local(const LevelGeom& g, const I3& bc, const I3& lc) {
    return I3{bc.x * g.bdim[0] + lc.x, bc.y * g.bdim[1] + lc.y, bc.z * g.bdim[2] + lc.z};
}

// Neighbour of local point lc of block bc: returns the local index when the
// (wrapped) neighbour lies inside the block, else -1; *glob receives its
// global index (-1 outside a Dirichlet grid).
__device__ __forceinline__ int block_neighbour(const LevelGeom& g, const I3& bc, const I3& lc, int ax, int d,
                                               int* glob) {
    I3 gi;
    const int gn = neighbour(g, global_of_local(g, bc, lc), ax, d, &gi);
    *glob = gn;
    if (gn < 0) return -1;
    const I3 ln{gi.x - bc.x * g.bdim[0], gi.y - bc.y * g.bdim[1], gi.z - bc.z * g.bdim[2]};
    if (ln.x < 0 || ln.x >= g.bdim[0] || ln.y < 0 || ln.y >= g.bdim[1] || ln.z < 0 || ln.z >= g.bdim[2]) return -1;
    return local_index(g, ln);
}

// ---------------------------------------------------------------------------
// reductions (deterministic: fixed thread -> element assignment, fixed tree)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup; the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double tot = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) tot += sh[k];
    __syncthreads();
    return tot;
}

// Sum over aligned groups of G consecutive lanes (G = 1, 2, 4 or 8), returned
// in every lane of the group: DPP moves within a quad (lanes ^ 1, ^ 2), then
// between the two quads of a group of eight (row_half_mirror).  Every lane of
// the wave must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1, 2, 4, 8 or 16 lanes");
    if constexpr (G >= 2) v += dpp_move<0xB1>(v);    // quad_perm (1, 0, 3, 2)
    if constexpr (G >= 4) v += dpp_move<0x4E>(v);    // quad_perm (2, 3, 0, 1)
    if constexpr (G >= 8) v += dpp_move<0x141>(v);   // row_half_mirror
    if constexpr (G >= 16) v += dpp_move<0x140>(v);  // row_mirror
    return v;
}

// Sum over the wave, the same value in every lane: the sums of the four rows of
// 16 lanes by DPP, then read from lanes 0, 16, 32 and 48 and added in that order.
// Every lane of the wave must be active.
__device__ __forceinline__ double wave_total(double v) {
    const long long u = __double_as_longlong(group_sum<16>(v));
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)u, 16 * r);
        const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), 16 * r);
        t += __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    }
    return t;
}

// The value of lane s of each quad (s < 4), in every lane of the quad.
template <typename T>
__device__ __forceinline__ cx<T> quad_bcast(const cx<T>& v, int s) {
    switch (s) {
        case 0: return cx<T>{dpp_move<0x00>(v.r), dpp_move<0x00>(v.i)};   // quad_perm (0, 0, 0, 0)
        case 1: return cx<T>{dpp_move<0x55>(v.r), dpp_move<0x55>(v.i)};   // quad_perm (1, 1, 1, 1)
        case 2: return cx<T>{dpp_move<0xAA>(v.r), dpp_move<0xAA>(v.i)};   // quad_perm (2, 2, 2, 2)
        default: return cx<T>{dpp_move<0xFF>(v.r), dpp_move<0xFF>(v.i)};  // quad_perm (3, 3, 3, 3)
    }
}

// ---------------------------------------------------------------------------
// K1: action residual of the step system (or its adjoint) + norm partials.
// One thread per (point, time component), kThreads / NT points per workgroup,
// so that every load and store of c and of the residual is contiguous across
// the wave; the workgroup stages its points' coefficients in LDS for the
// couplings between time components.
// ---------------------------------------------------------------------------
// Residual of item (point j, component m) of a group of points staged
// together: every thread of the workgroup calls it (it holds a barrier).
// cs holds the group's coefficients, slot = the thread's (point, m) position;
// cj points at the item's point in cs; tos (NT + NT^2 doubles of LDS) receives
// U and W, which are indexed per lane.  Returns rho_jm; for m == 0 also the
// constraint residual sigma_j (in *sg).
template <int NT>
__device__ __forceinline__ double2 residual_item(const LevelGeom& g, const TimeOps<NT>& to, int adjoint, int field_on,
                                                 const double2* __restrict__ c, const double2* __restrict__ lam,
                                                 const double* __restrict__ v0, const double2* __restrict__ bc,
                                                 const double2* __restrict__ bg, const double2* __restrict__ bs,
                                                 int j, int m, bool slot, double2* cs, int cslot, const double2* cj,
                                                 double* tos, double2* sg) {
    const I3 i = point_coords(g, j);
    const int t = threadIdx.x, iw = t - NT;
    const double tov = t < NT ? to.U[t] : to.W[(iw >= 0 && iw < NT * NT) ? iw : 0];
    const double2 own = c[(size_t)j * NT + m];
    // neighbour loads issued unconditionally (clamped index, 0/1 weight)
    int nbq[6];
    nbq[0] = neighbour_of<0, -1>(g, i, j);
    nbq[1] = neighbour_of<0, 1>(g, i, j);
    nbq[2] = g.dim > 1 ? neighbour_of<1, -1>(g, i, j) : -1;
    nbq[3] = g.dim > 1 ? neighbour_of<1, 1>(g, i, j) : -1;
    nbq[4] = g.dim > 2 ? neighbour_of<2, -1>(g, i, j) : -1;
    nbq[5] = g.dim > 2 ? neighbour_of<2, 1>(g, i, j) : -1;
    double2 nbv[6];
    double nbw[6];
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) {
        nbw[dir] = nbq[dir] >= 0 ? 1.0 : 0.0;
        nbv[dir] = c[(size_t)(nbq[dir] >= 0 ? nbq[dir] : j) * NT + m];
    }
    const double vj = v0[j];
    const double2 lj = lam[j];
    // optional right-hand sides loaded without branches (see k_sweep)
    const double2* rbp = bc ? bc + (size_t)j * NT + m : (bg ? bg + j : c + (size_t)j * NT + m);
    const double2 rhs = scl2((bc || bg) ? 1.0 : 0.0, *rbp);
    const double2 sgb = scl2((bs && m == 0) ? 1.0 : 0.0, (bs ? bs : lam)[j]);
    if (slot) cs[cslot] = own;
    if (t < NT + NT * NT) tos[t] = tov;
    __syncthreads();
    double2 lap = scl2(-2.0 * g.dim, own);
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) lap = add2(lap, scl2(nbw[dir], nbv[dir]));
    double2 tq = make_double2(0.0, 0.0);
    if (!adjoint) {
        for (int n = m + 1; n < NT; n += 2) tq = add2(tq, cj[n]);
    } else {
        for (int n = m - 1; n >= 0; n -= 2) tq = add2(tq, cj[n]);
    }
    // forward: i * 2 tq ; adjoint: -i * 2 tq
    const double2 tim = adjoint ? make_double2(2.0 * tq.y, -2.0 * tq.x) : make_double2(-2.0 * tq.y, 2.0 * tq.x);
    const double2 hc = add2(scl2(-g.kin, lap), scl2(vj, own));
    double2 row = sub2(tim, scl2(tos[m], hc));
    if (field_on) {
        double2 wc = make_double2(0.0, 0.0);
#pragma unroll
        for (int n = 0; n < NT; ++n) wc = add2(wc, scl2(tos[NT + m * NT + n], cj[n]));
        row = sub2(row, scl2(zcoord(g, i), wc));
    }
    row = add2(row, scl2((m & 1) ? -1.0 : 1.0, lj));
    if (m == 0) {
        double2 s = sgb;
#pragma unroll
        for (int n = 0; n < NT; ++n) s = (n & 1) ? add2(s, cj[n]) : sub2(s, cj[n]);
        *sg = s;
    }
    return sub2(rhs, row);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_residual(LevelGeom g, TimeOps<NT> to, int adjoint, int field_on,
                                                       const double2* __restrict__ c,
                                                       const double2* __restrict__ lam,
                                                       const double* __restrict__ v0,
                                                       const double2* __restrict__ bc,
                                                       const double2* __restrict__ bg,
                                                       const double2* __restrict__ bs,
                                                       double2* __restrict__ rc, double2* __restrict__ rs,
                                                       double* __restrict__ partial, const int* __restrict__ skip,
                                                       const unsigned char* __restrict__ bmask) {
    if (skip && *skip) return;
    constexpr int PW = kThreads / NT;  // points per workgroup
    __shared__ double2 cs[PW * NT];
    __shared__ double tos[NT + NT * NT];
    __shared__ double red[kThreads / 64];
    const int t = threadIdx.x;
    const int lp = t / NT, m = t - lp * NT;
    double acc = 0.0;
    const size_t jw = (size_t)blockIdx.x * PW + lp;
    const bool act = lp < PW && jw < (size_t)g.P;
    const int j = act ? (int)jw : 0;
    double2 sg = make_double2(0.0, 0.0);
    const double2 rho = residual_item<NT>(g, to, adjoint, field_on, c, lam, v0, bc, bg, bs, j, m, lp < PW, cs, t,
                                          cs + (lp < PW ? lp : 0) * NT, tos, &sg);
    if (act) {
        if (rc) rc[(size_t)j * NT + m] = rho;
        // bmask (one flag per subvolume): the norm counts the rows of flagged subvolumes only
        double wt = 1.0;
        if (bmask) {
            const I3 i = point_coords(g, j);
            wt = bmask[(i.x / g.bdim[0] * g.nblk[1] + i.y / g.bdim[1]) * g.nblk[2] + i.z / g.bdim[2]] ? 1.0 : 0.0;
        }
        acc += wt * tos[m] * (rho.x * rho.x + rho.y * rho.y);
        if (m == 0) {
            if (rs) rs[j] = sg;
            acc += wt * (sg.x * sg.x + sg.y * sg.y);
        }
    }
    if (partial) {
        const double tot = block_sum(acc, red);
        if (threadIdx.x == 0) partial[blockIdx.x] = tot;
    }
}

// K1+K4 fused: the residual of a level projected straight to the next coarser
// level (average of the 2^d children), without storing the fine residual;
// also clears the coarse correction.  A workgroup takes a tile of 32 fine
// points: 2 along every axis but the last, 32 / 2^(d-1) along the last, which
// holds whole child groups of 32 / 2^d coarse points.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_residual_restrict(LevelGeom f, LevelGeom cg, TimeOps<NT> to,
                                                                int adjoint, int field_on,
                                                                const double2* __restrict__ c,
                                                                const double2* __restrict__ lam,
                                                                const double* __restrict__ v0,
                                                                const double2* __restrict__ bc,
                                                                const double2* __restrict__ bg,
                                                                const double2* __restrict__ bs,
                                                                double2* __restrict__ bcc, double2* __restrict__ bsc,
                                                                double2* __restrict__ zc, double2* __restrict__ zl,
                                                                int t1, int t2, double rt1, double rt2) {
    // t1, t2: tile counts along axes 1 and 2 (rt1, rt2: their reciprocals)
    constexpr int PT = 32;
    constexpr int NQ = NT + 1;
    static_assert(PT * kMaxNT <= kThreads, "one item per thread");
    __shared__ double2 cs[PT * NT];
    __shared__ double2 rb[PT * NQ];
    __shared__ double tos[NT + NT * NT];
    const int t = threadIdx.x;
    const int lp = t / NT, m = t - lp * NT;
    const int dim = f.dim;
    const int sl = 6 - dim;                       // log2 of the tile extent along the last axis
    // tile extents (unused axes 1) and tile counts
    const int e0 = dim == 1 ? (1 << sl) : 2, e1 = dim == 1 ? 1 : (dim == 2 ? (1 << sl) : 2);
    const int e2 = dim == 3 ? (1 << sl) : 1;
    const int le1 = dim == 1 ? 0 : (dim == 2 ? sl : 1), le2 = dim == 3 ? sl : 0;  // log2 e1, log2 e2
    const int bid = (int)blockIdx.x;
    const int byx = qdiv(bid, rt2), bz = bid - byx * t2;
    const int bx = qdiv(byx, rt1), by = byx - bx * t1;
    // this thread's fine point
    const int lz = lp & (e2 - 1), ly = (lp >> le2) & (e1 - 1), lx = lp >> (le1 + le2);
    const I3 fi{bx * e0 + lx, by * e1 + ly, bz * e2 + lz};
    const bool inside = lp < PT && fi.x < f.n[0] && fi.y < f.n[1] && fi.z < f.n[2];
    const int j = inside ? point_index(f, fi) : 0;
    double2 sg = make_double2(0.0, 0.0);
    const double2 rho = residual_item<NT>(f, to, adjoint, field_on, c, lam, v0, bc, bg, bs, j, m, lp < PT, cs, t,
                                          cs + (lp < PT ? lp : 0) * NT, tos, &sg);
    if (lp < PT) {
        rb[lp * NQ + m] = rho;
        if (m == 0) rb[lp * NQ + NT] = sg;
    }
    __syncthreads();
    // coarse points of the tile: extents e/2 (1 on unused axes)
    const int c0 = dim == 1 ? e0 >> 1 : 1, c1 = dim == 2 ? e1 >> 1 : 1, c2 = dim == 3 ? e2 >> 1 : 1;
    const int ncp = c0 * c1 * c2;
    if (t < ncp * NQ) {
        const int cp = t / NQ, n = t - cp * NQ;
        const int lc1 = dim == 2 ? le1 - 1 : 0, lc2 = dim == 3 ? le2 - 1 : 0;  // log2 c1, log2 c2
        const int cz = cp & (c2 - 1), cy = (cp >> lc2) & (c1 - 1), cx = cp >> (lc1 + lc2);
        const I3 ci{(bx * e0 >> 1) + cx, (by * e1 >> 1) + cy, (bz * e2 >> 1) + cz};
        // with unused axes of extent 1 the formulas above give coordinate 0 there
        const I3 cc{dim >= 1 ? ci.x : 0, dim >= 2 ? ci.y : 0, dim >= 3 ? ci.z : 0};
        if (cc.x < cg.n[0] && cc.y < cg.n[1] && cc.z < cg.n[2]) {
            const int nch = 1 << dim;
            double2 acc = make_double2(0.0, 0.0);
            for (int ch = 0; ch < nch; ++ch) {
                // child (2 cx + s0, 2 cy + s1, 2 cz + s2) in tile-local coordinates, along used axes
                const int s0 = ch & 1, s1 = (ch >> 1) & 1, s2 = (ch >> 2) & 1;
                const int fx = dim >= 1 ? (dim == 1 ? 2 * cx + s0 : s0) : 0;
                const int fy = dim >= 2 ? (dim == 2 ? 2 * cy + s1 : s1) : 0;
                const int fz = dim == 3 ? 2 * cz + s2 : 0;
                acc = add2(acc, rb[((fx * e1 + fy) * e2 + fz) * NQ + n]);
            }
            acc = scl2(1.0 / nch, acc);
            const int J = point_index(cg, cc);
            if (n < NT) {
                bcc[(size_t)J * NT + n] = acc;
                zc[(size_t)J * NT + n] = make_double2(0.0, 0.0);
            } else {
                bsc[J] = acc;
                zl[J] = make_double2(0.0, 0.0);
            }
        }
    }
}

// K1 and K1+K4 on 3D levels: a workgroup takes an 8 x 8 tile of the (y, z)
// plane, four lanes per point (lane q holds the time components q and q + 4,
// like the pair sweep), and marches along x over a range of planes.  A point's
// neighbours across x stay in the registers of its lanes (previous, current and
// next plane); the current plane and its one-point halo in y and z sit in LDS
// (two buffers, one barrier per plane).  Each coefficient is read 1.5 times
// (own plane + halo) instead of once per stencil neighbour, and the work of a
// point (addresses, potential, multiplier, right-hand sides, the constraint
// row) is shared by its two components.  The arithmetic of each item is that
// of residual_item (the constraint sum taken over the point's lanes);
// RESTRICT: the residual is averaged over the 2 x 2 x 2 children of each
// coarse point (planes 2X and 2X + 1 of the range) as in k_residual_restrict,
// else the norm partial of the workgroup.
constexpr int kMarchTY = 8, kMarchTZ = 8;

template <int NT, bool RESTRICT>
__global__ __launch_bounds__(kThreads, 3) void k_residual_march(
    LevelGeom g, LevelGeom cg, TimeOps<NT> to, int adjoint, int field_on, const double2* __restrict__ c,
    const double2* __restrict__ lam, const double* __restrict__ v0, const double2* __restrict__ bc,
    const double2* __restrict__ bg, const double2* __restrict__ bs, double2* __restrict__ rc,
    double2* __restrict__ rs, double* __restrict__ partial, const int* __restrict__ skip,
    const unsigned char* __restrict__ bmask, double2* __restrict__ bcc, double2* __restrict__ bsc,
    double2* __restrict__ zc, double2* __restrict__ zl, int tiles_y, int tiles_z, int xs) {
    if (skip && *skip) return;
    constexpr int TY = kMarchTY, TZ = kMarchTZ, HZ = TZ + 2, HP = (TY + 2) * HZ;
    constexpr int NQ = NT + 1, IPL = 2;
    // LDS slot stride of a point: odd in units of 16 bytes, so that the 16 points of
    // a wave reading one component spread over the banks (an even stride puts
    // them in a few bank groups)
    constexpr int NTP = NT | 1;
    constexpr int NHALO = 2 * TZ + 2 * TY;   // halo points of a plane tile (no corners)
    static_assert(TY * TZ * 4 == kThreads && NHALO * 8 == kThreads, "four lanes per point, one halo item per thread");
    __shared__ double2 pl[2][HP * NTP];
    __shared__ double2 rb[RESTRICT ? 2 : 1][RESTRICT ? TY * TZ * NQ : 1];
    __shared__ double tos[NT + NT * NT];
    __shared__ double red[kThreads / 64];
    const int t = threadIdx.x;
    const int q = t & 3, pz = (t >> 2) & (TZ - 1), py = t >> 5;
    bool item[IPL];
    int mi[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        item[k] = q + 4 * k < NT;
        mi[k] = item[k] ? q + 4 * k : 0;
    }
    const int bid = (int)blockIdx.x;
    const int q0 = bid / tiles_z, tzi = bid - q0 * tiles_z;
    const int xr = q0 / tiles_y, tyi = q0 - xr * tiles_y;
    const int n0 = g.n[0], n1 = g.n[1], n2 = g.n[2];
    const size_t sx = (size_t)n1 * n2;
    const int y = tyi * TY + py, z = tzi * TZ + pz;
    const int jyz = y * n2 + z;
    const int x0 = xr * xs, x1 = min(n0, x0 + xs);
    // this thread's halo item: point hp of the halo ring, component hm
    const int hp = t >> 3, hm = t & 7;
    int hy, hz;
    if (hp < TZ) { hy = -1; hz = hp; }
    else if (hp < 2 * TZ) { hy = TY; hz = hp - TZ; }
    else if (hp < 2 * TZ + TY) { hy = hp - 2 * TZ; hz = -1; }
    else { hy = hp - 2 * TZ - TY; hz = TZ; }
    int gy = tyi * TY + hy, gz = tzi * TZ + hz;
    bool hval = hm < NT;
    if (gy < 0 || gy >= n1) { gy += gy < 0 ? n1 : -n1; hval = hval && g.periodic; }
    if (gz < 0 || gz >= n2) { gz += gz < 0 ? n2 : -n2; hval = hval && g.periodic; }
    const int hmc = hm < NT ? hm : 0;
    const int hj = gy * n2 + gz;
    const int hslot = ((hy + 1) * HZ + (hz + 1)) * NTP + hmc;
    const int oslot = ((py + 1) * HZ + (pz + 1)) * NTP;
    // plane x (one past either end: wrapped, or zero under Dirichlet)
    auto plane = [&](int x, bool& ok) {
        ok = true;
        if (x < 0) { x += n0; ok = g.periodic; }
        else if (x >= n0) { x -= n0; ok = g.periodic; }
        return x;
    };
    auto load_own = [&](int x, double2* v) {
        bool ok;
        const int xx = plane(x, ok);
        const double2* src = c + ((size_t)xx * sx + jyz) * NT;
#pragma unroll
        for (int k = 0; k < IPL; ++k) v[k] = scl2(ok && item[k] ? 1.0 : 0.0, src[mi[k]]);
    };
    auto load_halo = [&](int x) {
        bool ok;
        const int xx = plane(x, ok);
        return scl2(ok && hval ? 1.0 : 0.0, c[((size_t)xx * sx + hj) * NT + hmc]);
    };
    if (t < NT + NT * NT) tos[t] = t < NT ? to.U[t] : to.W[t - NT];
    double2 cprev[IPL], ccur[IPL], cnext[IPL];
    load_own(x0 - 1, cprev);
    load_own(x0, ccur);
    {
        const double2 h0 = load_halo(x0);
#pragma unroll
        for (int k = 0; k < IPL; ++k)
            if (item[k]) pl[0][oslot + mi[k]] = ccur[k];
        if (hm < NT) pl[0][hslot] = h0;
    }
    __syncthreads();
    double u_m[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) u_m[k] = tos[mi[k]];
    double acc = 0.0;
    double2 cacc = make_double2(0.0, 0.0);
    for (int x = x0; x < x1; ++x) {
        const int b = (x - x0) & 1;
        // the next plane, and this plane's point data
        load_own(x + 1, cnext);
        const double2 hnext = load_halo(x + 1);
        const size_t j = (size_t)x * sx + jyz;
        const double vj = v0[j];
        const double2 lj = lam[j];
        double2 rhs[IPL];
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            const double2* rbp = bc ? bc + j * NT + mi[k] : (bg ? bg + j : c + j * NT + mi[k]);
            rhs[k] = scl2((bc || bg) ? 1.0 : 0.0, *rbp);
        }
        const double2 sgb = scl2(bs ? 1.0 : 0.0, (bs ? bs : lam)[j]);
        const double2* P = pl[b] + oslot;
        // the constraint residual of the point: bs - sum_n (-1)^n c_n over its lanes
        double2 sg;
        {
            double2 part = make_double2(0.0, 0.0);
#pragma unroll
            for (int k = 0; k < IPL; ++k)
                part = add2(part, scl2(item[k] ? ((mi[k] & 1) ? 1.0 : -1.0) : 0.0, ccur[k]));
            sg = add2(sgb, make_double2(group_sum<4>(part.x), group_sum<4>(part.y)));
        }
        const double zf = field_on ? zcoord(g, I3{x, y, z}) : 0.0;
        double2 rho[IPL];
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            const int m = mi[k];
            double2 lap = add2(scl2(-6.0, ccur[k]), add2(cprev[k], cnext[k]));
            lap = add2(lap, add2(P[-HZ * NTP + m], P[HZ * NTP + m]));
            lap = add2(lap, add2(P[-NTP + m], P[NTP + m]));
            double2 tq = make_double2(0.0, 0.0);
#pragma unroll
            for (int kk = 0; kk < (NT + 1) / 2; ++kk) {
                const int n = adjoint ? m - 1 - 2 * kk : m + 1 + 2 * kk;
                const bool in = n >= 0 && n < NT;
                tq = add2(tq, scl2(in ? 1.0 : 0.0, P[in ? n : m]));
            }
            const double2 tim = adjoint ? make_double2(2.0 * tq.y, -2.0 * tq.x) : make_double2(-2.0 * tq.y, 2.0 * tq.x);
            const double2 hc = add2(scl2(-g.kin, lap), scl2(vj, ccur[k]));
            double2 row = sub2(tim, scl2(u_m[k], hc));
            if (field_on) {
                double2 wc = make_double2(0.0, 0.0);
#pragma unroll
                for (int n = 0; n < NT; ++n) wc = add2(wc, scl2(tos[NT + m * NT + n], P[n]));
                row = sub2(row, scl2(zf, wc));
            }
            row = add2(row, scl2((m & 1) ? -1.0 : 1.0, lj));
            rho[k] = sub2(rhs[k], row);
        }
        if constexpr (RESTRICT) {
            double2* R = rb[b] + (py * TZ + pz) * NQ;
#pragma unroll
            for (int k = 0; k < IPL; ++k)
                if (item[k]) R[mi[k]] = rho[k];
            if (q == 0) R[NT] = sg;
        } else {
            double wt = 1.0;
            if (bmask)
                wt = bmask[((x / g.bdim[0]) * g.nblk[1] + y / g.bdim[1]) * g.nblk[2] + z / g.bdim[2]] ? 1.0 : 0.0;
#pragma unroll
            for (int k = 0; k < IPL; ++k) {
                if (!item[k]) continue;
                if (rc) rc[j * NT + mi[k]] = rho[k];
                acc += wt * u_m[k] * (rho[k].x * rho[k].x + rho[k].y * rho[k].y);
            }
            if (q == 0) {
                if (rs) rs[j] = sg;
                acc += wt * (sg.x * sg.x + sg.y * sg.y);
            }
        }
        // the next plane into the other buffer
#pragma unroll
        for (int k = 0; k < IPL; ++k)
            if (item[k]) pl[b ^ 1][oslot + mi[k]] = cnext[k];
        if (hm < NT) pl[b ^ 1][hslot] = hnext;
        __syncthreads();
        if constexpr (RESTRICT) {
            // coarse points of the tile: 4 x 4, NQ values each (threads < 16 NQ)
            if (t < (TY / 2) * (TZ / 2) * NQ) {
                const int cp = t / NQ, qq = t - cp * NQ;
                const int cy = cp / (TZ / 2), cz = cp - cy * (TZ / 2);
                const double2* R = rb[b];
                double2 s4 = add2(R[((2 * cy) * TZ + 2 * cz) * NQ + qq], R[((2 * cy) * TZ + 2 * cz + 1) * NQ + qq]);
                s4 = add2(s4, add2(R[((2 * cy + 1) * TZ + 2 * cz) * NQ + qq], R[((2 * cy + 1) * TZ + 2 * cz + 1) * NQ + qq]));
                cacc = add2(cacc, s4);
                if (x & 1) {
                    const int J = ((x >> 1) * cg.n[1] + (tyi * TY >> 1) + cy) * cg.n[2] + (tzi * TZ >> 1) + cz;
                    const double2 v = scl2(0.125, cacc);
                    if (qq < NT) {
                        bcc[(size_t)J * NT + qq] = v;
                        zc[(size_t)J * NT + qq] = make_double2(0.0, 0.0);
                    } else {
                        bsc[J] = v;
                        zl[J] = make_double2(0.0, 0.0);
                    }
                    cacc = make_double2(0.0, 0.0);
                }
            }
        }
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            cprev[k] = ccur[k];
            ccur[k] = cnext[k];
        }
    }
    if constexpr (!RESTRICT) {
        if (partial) {
            const double tot = block_sum(acc, red);
            if (t == 0) partial[bid] = tot;
        }
    }
}

// Whether a level takes the marching residual: 3D, the (y, z) plane tiled by
// 8 x 8 exactly and an even x extent (pairs of planes restrict together).
// Planes per workgroup: long ranges on large levels, short ones on small levels
// (enough workgroups to fill the device).
inline bool march_fits(const LevelGeom& g) {
    return g.dim == 3 && g.n[1] % kMarchTY == 0 && g.n[2] % kMarchTZ == 0 && g.n[0] % 2 == 0;
}
inline int march_planes(const LevelGeom& g) { return g.n[0] >= 128 ? 16 : (g.n[0] >= 32 ? 8 : 2); }
inline int march_blocks(const LevelGeom& g) {
    const int xs = march_planes(g);
    return (g.n[1] / kMarchTY) * (g.n[2] / kMarchTZ) * ((g.n[0] + xs - 1) / xs);
}

// Sum of the partials in a fixed order (one 1024-thread workgroup, four
// independent accumulators per thread so the loads stay in flight).
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void k_reduce(const double* __restrict__ partial, int nparts,
                                                           double* __restrict__ out) {
    __shared__ double red[kReduceThreads / 64];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int k = threadIdx.x;
    for (; k + 3 * kReduceThreads < nparts; k += 4 * kReduceThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += partial[k + u * kReduceThreads];
    }
    for (; k < nparts; k += kReduceThreads) acc[0] += partial[k];
    const double tot = block_sum((acc[0] + acc[1]) + (acc[2] + acc[3]), red);
    if (threadIdx.x == 0) out[0] = tot;
}

// The same sum, closing one step of the iterated coarsest-level solve (see
// launch_reduce_ctl).
__global__ __launch_bounds__(kReduceThreads) void k_reduce_ctl(const double* __restrict__ partial, int nparts,
                                                               CoarseCtl* __restrict__ ctl, int start, double thr2,
                                                               int* __restrict__ iters_out) {
    __shared__ double red[kReduceThreads / 64];
    if (!start && ctl->done) {
        if (threadIdx.x == 0 && iters_out) *iters_out = ctl->iters | (1 << 30);
        return;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int k = threadIdx.x;
    for (; k + 3 * kReduceThreads < nparts; k += 4 * kReduceThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += partial[k + u * kReduceThreads];
    }
    for (; k < nparts; k += kReduceThreads) acc[0] += partial[k];
    const double tot = block_sum((acc[0] + acc[1]) + (acc[2] + acc[3]), red);
    if (threadIdx.x == 0) {
        if (start) {
            ctl->n0 = tot;
            ctl->n = tot;
            ctl->done = tot == 0.0 ? 1 : 0;
            ctl->iters = 0;
        } else {
            ctl->iters += 1;
            ctl->n = tot;
            ctl->done = tot <= thr2 * ctl->n0 ? 1 : 0;
        }
        if (iters_out) *iters_out = ctl->iters | (ctl->done ? (1 << 30) : 0);
    }
}

// One workgroup per output element w: out[w] = sum_p partial[p * width + w].
__global__ __launch_bounds__(kThreads) void k_reduce_c2(const double2* __restrict__ partial, int nparts,
                                                        int width, double2* __restrict__ out) {
    __shared__ double red[kThreads / 64];
    const int w = blockIdx.x;
    double ar = 0.0, ai = 0.0;
    for (int k = threadIdx.x; k < nparts; k += kThreads) {
        const double2 v = partial[(size_t)k * width + w];
        ar += v.x;
        ai += v.y;
    }
    const double tr = block_sum(ar, red);
    const double ti = block_sum(ai, red);
    if (threadIdx.x == 0) out[w] = make_double2(tr, ti);
}

// ---------------------------------------------------------------------------
// K4: projection of a residual to the next level (average of the 2^d
// children); also clears the coarse correction.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(kThreads) void k_restrict(LevelGeom f, LevelGeom cg,
                                                       const double2* __restrict__ rcf,
                                                       const double2* __restrict__ rsf,
                                                       double2* __restrict__ bcc, double2* __restrict__ bsc,
                                                       double2* __restrict__ zc, double2* __restrict__ zl) {
    // one thread per (coarse point, component): components 0..NT-1 of c, then lambda
    constexpr int NQ = NT + 1;
    const size_t t = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (t >= (size_t)cg.P * NQ) return;
    const int J = (int)(t / NQ), n = (int)(t - (size_t)J * NQ);
    const bool isc = n < NT;
    const double2* src = isc ? rcf + n : rsf;
    const int stride = isc ? NT : 1;
    const I3 I = point_coords(cg, J);
    const int nch = 1 << f.dim;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int ch = 0; ch < 8; ++ch) {
        const int chc = ch < nch ? ch : 0;
        const double w = ch < nch ? 1.0 : 0.0;
        // child offsets only along the grid's axes (unused axes have extent 1)
        const I3 fi{2 * I.x + ((chc >> 0) & 1), f.dim > 1 ? 2 * I.y + ((chc >> 1) & 1) : 0,
                    f.dim > 2 ? 2 * I.z + ((chc >> 2) & 1) : 0};
        acc = add2(acc, scl2(w, src[(size_t)point_index(f, fi) * stride]));
    }
    acc = scl2(1.0 / nch, acc);
    if (isc) {
        bcc[(size_t)J * NT + n] = acc;
        if (zc) zc[(size_t)J * NT + n] = make_double2(0.0, 0.0);
    } else {
        bsc[J] = acc;
        if (zl) zl[J] = make_double2(0.0, 0.0);
    }
}

// Partials of N of a right-hand side held as (rho, sigma) rows, sum_j sum_m U_m
// |rho_jm|^2 + |sigma_j|^2 (the projected residual of the adaptive tree's
// composite norm), laid out as k_residual's partials.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_rhs_norm(int P, TimeOps<NT> to, const double2* __restrict__ rho,
                                                       const double2* __restrict__ sig, double* __restrict__ partial) {
    constexpr int PW = kThreads / NT;
    __shared__ double red[kThreads / 64];
    const int t = threadIdx.x;
    const int lp = t / NT, m = t - lp * NT;
    const size_t j = (size_t)blockIdx.x * PW + lp;
    double acc = 0.0;
    if (lp < PW && j < (size_t)P) {
        const double2 r = rho[j * NT + m];
        double u = to.U[0];
#pragma unroll
        for (int k = 1; k < NT; ++k) u = m == k ? to.U[k] : u;
        acc = u * (r.x * r.x + r.y * r.y);
        if (m == 0) {
            const double2 q = sig[j];
            acc += q.x * q.x + q.y * q.y;
        }
    }
    const double tot = block_sum(acc, red);
    if (t == 0) partial[blockIdx.x] = tot;
}

// Haar detail energy per subvolume (one 64-lane workgroup each): sum over its
// points j of |psi_j - mean of psi over the 2^d children of j's parent cell|^2,
// reduced in a fixed order.
__global__ __launch_bounds__(64) void k_block_detail(LevelGeom g, const double2* __restrict__ psi,
                                                     double* __restrict__ out) {
    const int blk = blockIdx.x, l = threadIdx.x;
    double d = 0.0;
    if (l < g.bpts) {
        const I3 bc = block_coords(g, blk);
        const I3 i = global_of_local(g, bc, local_coords(g, l));
        const int nch = 1 << g.dim;
        double2 mean = make_double2(0.0, 0.0);
        for (int ch = 0; ch < nch; ++ch) {
            const I3 s{(i.x & ~1) | (ch & 1), g.dim > 1 ? ((i.y & ~1) | ((ch >> 1) & 1)) : 0,
                       g.dim > 2 ? ((i.z & ~1) | ((ch >> 2) & 1)) : 0};
            mean = add2(mean, psi[point_index(g, s)]);
        }
        const double2 p = psi[point_index(g, i)];
        const double dr = p.x - mean.x / nch, di = p.y - mean.y / nch;
        d = dr * dr + di * di;
    }
    d = wave_sum(d);
    if (l == 0) out[blk] = d;
}

// ---------------------------------------------------------------------------
// K5: interpolation of a coarse correction, added into the fine state,
// c_f += I c_c and lambda_f += I lambda_c (Sec. "Multigrid Relaxation", Eq.
// (correction_fine)).  interp 0: cell-centred tensor-linear (3/4 parent, 1/4
// nearer neighbour per axis; zero outside a Dirichlet grid); 1: piecewise
// constant.
// A workgroup takes a coarse tile of 2 x 2 x 8 points (2 along the used axes
// but the last, 8 along the last; 1 along unused axes), stages it with a
// one-point coarse halo in LDS (every component, zero outside a Dirichlet
// grid, wrapped on a periodic one), and adds the interpolated correction to
// the fine tile of its children.  Each coarse value is read from memory by
// the few tiles whose halo holds it, instead of by every fine point that
// interpolates from it.
// ---------------------------------------------------------------------------
template <int NT, int D>
__global__ __launch_bounds__(kThreads) void k_prolong_tile(LevelGeom f, LevelGeom cg, int interp,
                                                           const double2* __restrict__ cc,
                                                           const double2* __restrict__ lc,
                                                           double2* __restrict__ cf, double2* __restrict__ lf,
                                                           int t1, int t2) {
    constexpr int NQ = NT + 1;
    constexpr int HMAX = 4 * 4 * 10;                 // halo points of a 3D tile
    __shared__ double2 S[HMAX * NQ];
    // D > 0: the rank at compile time (tile extents and the index quotients below
    // become constants); D = 0: the level's rank
    const int dim = D > 0 ? D : f.dim;
    // coarse tile extents and the tile's first coarse point
    const int ct0 = dim == 1 ? 8 : 2, ct1 = dim == 1 ? 1 : (dim == 2 ? 8 : 2), ct2 = dim == 3 ? 8 : 1;
    const int bid = (int)blockIdx.x;
    const int bxy = bid / t2, bz = bid - bxy * t2;
    const int bx = bxy / t1, by = bxy - bx * t1;
    const I3 c0{bx * ct0, by * ct1, bz * ct2};
    // halo extents (one more coarse point on each side of a used axis)
    const int h0 = ct0 + 2, h1 = dim > 1 ? ct1 + 2 : 1, h2 = dim > 2 ? ct2 + 2 : 1;
    const int H = h0 * h1 * h2;
    for (int t = threadIdx.x; t < H * NQ; t += kThreads) {
        const int hp = t / NQ, q = t - hp * NQ;
        const int hz = hp % h2, hxy = hp / h2, hy = hxy % h1, hx = hxy / h1;
        // coarse coordinates of the halo point (axes beyond the rank have extent 1)
        int cx = c0.x + hx - 1, cy = dim > 1 ? c0.y + hy - 1 : 0, cz = dim > 2 ? c0.z + hz - 1 : 0;
        bool in = true;
        // (halo points past a partial tile that no fine point uses may lie more than
        // one grid length away: reduce fully, so that every load stays in the grid)
        auto fold = [&](int& v, int n) {
            if (v < 0 || v >= n) {
                if (f.periodic) v = ((v % n) + n) % n;
                else in = false;
            }
        };
        fold(cx, cg.n[0]);
        fold(cy, cg.n[1]);
        fold(cz, cg.n[2]);
        double2 v = make_double2(0.0, 0.0);
        if (in) {
            const int J = (cx * cg.n[1] + cy) * cg.n[2] + cz;
            v = q < NT ? cc[(size_t)J * NT + q] : lc[J];
        }
        S[t] = v;
    }
    __syncthreads();
    // fine tile: the children of the coarse tile
    const int f0 = dim >= 1 ? 2 * ct0 : 1, f1 = dim >= 2 ? 2 * ct1 : 1, f2 = dim >= 3 ? 2 * ct2 : 1;
    const int F = f0 * f1 * f2;
    for (int t = threadIdx.x; t < F * NQ; t += kThreads) {
        const int fp = t / NQ, q = t - fp * NQ;
        const int lz = fp % f2, lxy = fp / f2, ly = lxy % f1, lx = lxy / f1;
        const I3 fi{2 * c0.x + lx, dim > 1 ? 2 * c0.y + ly : 0, dim > 2 ? 2 * c0.z + lz : 0};
        if (fi.x >= f.n[0] || fi.y >= f.n[1] || fi.z >= f.n[2]) continue;
        // per axis: the parent's halo coordinate, the step to the nearer coarse
        // neighbour and the two weights (linear: 3/4 and 1/4; constant: 1 and 0)
        int hp[3], hd[3];
        double w0[3], w1[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int ia = comp(fi, a);
            const bool used = a < dim;
            hp[a] = used ? (ia >> 1) - comp(c0, a) + 1 : 0;
            hd[a] = used ? ((ia & 1) ? 1 : -1) : 0;
            const bool lin = !interp && used;
            w0[a] = lin ? 0.75 : 1.0;
            w1[a] = lin ? 0.25 : 0.0;
        }
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int cmb = 0; cmb < 8; ++cmb) {
            const int x = hp[0] + ((cmb & 1) ? hd[0] : 0), y = hp[1] + ((cmb & 2) ? hd[1] : 0),
                      z = hp[2] + ((cmb & 4) ? hd[2] : 0);
            const double w = ((cmb & 1) ? w1[0] : w0[0]) * ((cmb & 2) ? w1[1] : w0[1]) * ((cmb & 4) ? w1[2] : w0[2]);
            acc = add2(acc, scl2(w, S[((x * h1 + y) * h2 + z) * NQ + q]));
        }
        const int j = point_index(f, fi);
        double2* dst = q < NT ? cf + (size_t)j * NT + q : lf + j;
        *dst = add2(*dst, acc);
    }
}

__global__ __launch_bounds__(kThreads) void k_average_potential(LevelGeom f, LevelGeom cg,
                                                                const double* __restrict__ vf,
                                                                double* __restrict__ vc) {
    const int J = blockIdx.x * kThreads + threadIdx.x;
    if (J >= cg.P) return;
    const I3 I = point_coords(cg, J);
    const int nch = 1 << f.dim;
    double acc = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
        const I3 fi{2 * I.x + (ch & 1), f.dim > 1 ? 2 * I.y + ((ch >> 1) & 1) : 0,
                    f.dim > 2 ? 2 * I.z + ((ch >> 2) & 1) : 0};
        acc += vf[point_index(f, fi)];
    }
    vc[J] = acc / nch;
}

// ---------------------------------------------------------------------------
// K2a: spectral factor of every block's spatial operator A_U = T_U + diag(V0_U)
// (T_U: the kinetic stencil restricted to the block, exterior fixed at zero).
// Parallel cyclic Jacobi in LDS, one 512-thread workgroup per block, with the
// round-robin pairing: each round rotates nn/2 disjoint index pairs (p_i, q_i)
// at once, A <- G A G^T and V <- V G^T with G the direct sum of the 2 x 2
// rotations.  The two-sided update is done in one pass over 2 x 2 blocks
// (rows {p_i, q_i}, columns {p_j, q_j}), so a round has two barriers.
// Output V[blk][point][mode], e[blk][mode].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kSweepThreads) void k_block_eig(LevelGeom g, const double* __restrict__ v0,
                                                             double* __restrict__ Vout, double* __restrict__ eout,
                                                             float* __restrict__ Vfout) {
    __shared__ double A[kMaxB * kLdsPad];
    __shared__ double V[kMaxB * kLdsPad];
    __shared__ double rot_c[kMaxB / 2 + 1], rot_s[kMaxB / 2 + 1];
    __shared__ int rot_p[kMaxB / 2 + 1], rot_q[kMaxB / 2 + 1];
    __shared__ double red[kSweepThreads / 64];
    __shared__ int stop;

    const int tid = threadIdx.x;
    const int blk = blockIdx.x;
    const int b = g.bpts;
    const int nn = b + (b & 1);
    const int half = nn / 2;
    const float rhalf = 1.0f / (float)half;
    const I3 bc = block_coords(g, blk);

    for (int t = tid; t < b * b; t += kSweepThreads) {
        const int j = qdiv_small(t, g.rbp), k = t - j * b;
        A[j * kLdsPad + k] = 0.0;
        V[j * kLdsPad + k] = (j == k) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int l = tid; l < b; l += kSweepThreads) {
        const I3 lc = local_coords(g, l);
        A[l * kLdsPad + l] += 2.0 * g.dim * g.kin + v0[point_index(g, global_of_local(g, bc, lc))];
        for (int ax = 0; ax < g.dim; ++ax)
            for (int d = -1; d <= 1; d += 2) {
                int glob;
                const int ln = block_neighbour(g, bc, lc, ax, d, &glob);
                if (ln >= 0) A[l * kLdsPad + ln] += -g.kin;
            }
    }
    __syncthreads();

    for (int sweep = 0; sweep < 40; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int t = tid; t < b * b; t += kSweepThreads) {
            const int j = qdiv_small(t, g.rbp), k = t - j * b;
            const double v = A[j * kLdsPad + k];
            tot += v * v;
            if (j != k) off += v * v;
        }
        off = block_sum(off, red);
        tot = block_sum(tot, red);
        // off-diagonal Frobenius norm below 1e-14 of the total: at the level
        // the rotations themselves leave, so further sweeps cannot lower it
        if (tid == 0) stop = (off <= 1e-28 * tot) ? 1 : 0;
        __syncthreads();
        if (stop) break;
        for (int r = 0; r < nn - 1; ++r) {
            if (tid < half) {
                // round r of the round-robin: pair 0 = (r, nn-1), pair i = (r+i, r-i) mod nn-1
                int p = tid == 0 ? r : r + tid, q = tid == 0 ? nn - 1 : r - tid;
                if (tid != 0) {
                    p -= p >= nn - 1 ? nn - 1 : 0;
                    q += q < 0 ? nn - 1 : 0;
                }
                if (p > q) {
                    const int tmp = p;
                    p = q;
                    q = tmp;
                }
                double cth = 1.0, sth = 0.0;
                if (q < b) {
                    const double apq = A[p * kLdsPad + q];
                    if (fabs(apq) > 1e-300) {
                        const double tau = (A[q * kLdsPad + q] - A[p * kLdsPad + p]) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        cth = 1.0 / sqrt(1.0 + t * t);
                        sth = t * cth;
                    }
                }
                rot_p[tid] = p;
                rot_q[tid] = q < b ? q : p;   // a dummy pair (odd b) rotates nothing
                rot_c[tid] = cth;
                rot_s[tid] = q < b ? sth : 0.0;
            }
            __syncthreads();
            // A <- G A G^T on 2 x 2 blocks: rows (p_i, q_i), columns (p_j, q_j)
            for (int t = tid; t < half * half; t += kSweepThreads) {
                const int i = qdiv_small(t, rhalf), j = t - i * half;
                const int pi = rot_p[i], qi = rot_q[i], pj = rot_p[j], qj = rot_q[j];
                if (qi == pi && qj == pj) continue;  // both dummies: nothing to rotate
                const double ci = rot_c[i], si = rot_s[i], cj = rot_c[j], sj = rot_s[j];
                const double a00 = A[pi * kLdsPad + pj], a01 = A[pi * kLdsPad + qj];
                const double a10 = A[qi * kLdsPad + pj], a11 = A[qi * kLdsPad + qj];
                // rows: (p, q) <- (c p - s q, s p + c q)
                const double r00 = ci * a00 - si * a10, r01 = ci * a01 - si * a11;
                const double r10 = si * a00 + ci * a10, r11 = si * a01 + ci * a11;
                // columns: (p, q) <- (c p - s q, s p + c q)
                const double n00 = cj * r00 - sj * r01, n01 = sj * r00 + cj * r01;
                const double n10 = cj * r10 - sj * r11, n11 = sj * r10 + cj * r11;
                A[pi * kLdsPad + pj] = n00;
                if (qj != pj) A[pi * kLdsPad + qj] = n01;
                if (qi != pi) A[qi * kLdsPad + pj] = n10;
                if (qi != pi && qj != pj) A[qi * kLdsPad + qj] = n11;
            }
            // V <- V G^T: columns (p_j, q_j) of every row
            for (int t = tid; t < b * half; t += kSweepThreads) {
                const int k = qdiv_small(t, rhalf), j = t - k * half;
                const int pj = rot_p[j], qj = rot_q[j];
                if (qj == pj) continue;
                const double cj = rot_c[j], sj = rot_s[j];
                const double vp = V[k * kLdsPad + pj], vq = V[k * kLdsPad + qj];
                V[k * kLdsPad + pj] = cj * vp - sj * vq;
                V[k * kLdsPad + qj] = sj * vp + cj * vq;
            }
            __syncthreads();
        }
    }
    double* Vb = Vout + (size_t)blk * b * b;
    for (int t = tid; t < b * b; t += kSweepThreads) {
        const int j = qdiv_small(t, g.rbp), k = t - j * b;
        const double v = V[j * kLdsPad + k];
        Vb[t] = v;
        if (Vfout) Vfout[(size_t)blk * b * b + t] = (float)v;
    }
    for (int k = tid; k < b; k += kSweepThreads) eout[(size_t)blk * b + k] = A[k * kLdsPad + k];
}

// ---------------------------------------------------------------------------
// K2b: per block and mode, invert the time system of eigenvalue e,
//   M(e) = [[ iQ^T - e U - zf W, s ], [ s^T, 0 ]],  s_n = (-1)^n,
// (zf: the dipole coordinate of the block's slab record; W = 0 without field)
// by in-place Gauss-Jordan with partial pivoting.  One thread per mode; the
// matrix lives in LDS, interleaved across the 64 threads of the workgroup.
// ---------------------------------------------------------------------------
template <int NT>
__global__ __launch_bounds__(64) void k_mode_factor(LevelGeom g, TimeOps<NT> to, const double* __restrict__ e,
                                                    const double* __restrict__ tf, int tf_stride,
                                                    double2* __restrict__ Minv, float2* __restrict__ Minvf) {
    constexpr int NQ = NT + 1;
    __shared__ double2 M[NQ * NQ * 64];
    const int blk = blockIdx.x;
    const int k = threadIdx.x;
    const int b = g.bpts;
    if (k >= b) return;
    const double ev = e[(size_t)blk * b + k];
    const double zf = tf ? tf[(size_t)comp(block_coords(g, blk), g.fax) * tf_stride + tf_record_reals(NT)] : 0.0;
#define MAT(r, cc) M[((r) * NQ + (cc)) * 64 + k]
    for (int m = 0; m < NQ; ++m)
        for (int n = 0; n < NQ; ++n) {
            double2 v = make_double2(0.0, 0.0);
            if (m < NT && n < NT) {
                if (n > m && ((n - m) & 1)) v.y = 2.0;  // i Q_nm
                v.x = -zf * to.W[m * NT + n];
                if (m == n) v.x -= ev * to.U[m];
            } else if (m < NT && n == NT) {
                v.x = (m & 1) ? -1.0 : 1.0;
            } else if (m == NT && n < NT) {
                v.x = (n & 1) ? -1.0 : 1.0;
            }
            MAT(m, n) = v;
        }
    int piv[NQ];
    for (int col = 0; col < NQ; ++col) {
        int p = col;
        double best = -1.0;
        for (int r = col; r < NQ; ++r) {
            const double2 v = MAT(r, col);
            const double a = v.x * v.x + v.y * v.y;
            if (a > best) {
                best = a;
                p = r;
            }
        }
        piv[col] = p;
        if (p != col)
            for (int n = 0; n < NQ; ++n) {
                const double2 t = MAT(col, n);
                MAT(col, n) = MAT(p, n);
                MAT(p, n) = t;
            }
        const double2 d = MAT(col, col);
        const double den = d.x * d.x + d.y * d.y;
        const double2 inv = make_double2(d.x / den, -d.y / den);
        MAT(col, col) = make_double2(1.0, 0.0);
        for (int n = 0; n < NQ; ++n) {
            const double2 v = MAT(col, n);
            MAT(col, n) = make_double2(v.x * inv.x - v.y * inv.y, v.x * inv.y + v.y * inv.x);
        }
        for (int r = 0; r < NQ; ++r) {
            if (r == col) continue;
            const double2 f = MAT(r, col);
            MAT(r, col) = make_double2(0.0, 0.0);
            for (int n = 0; n < NQ; ++n) {
                const double2 a = MAT(col, n);
                const double2 v = MAT(r, n);
                MAT(r, n) = make_double2(v.x - (f.x * a.x - f.y * a.y), v.y - (f.x * a.y + f.y * a.x));
            }
        }
    }
    for (int col = NQ - 1; col >= 0; --col) {
        const int p = piv[col];
        if (p != col)
            for (int r = 0; r < NQ; ++r) {
                const double2 t = MAT(r, col);
                MAT(r, col) = MAT(r, p);
                MAT(r, p) = t;
            }
    }
    for (int p = 0; p < NQ; ++p)
        for (int q = 0; q < NQ; ++q) {
            const size_t o = (((size_t)blk * NQ + p) * NQ + q) * b + k;
            const double2 v = MAT(p, q);
            Minv[o] = v;
            if (Minvf) Minvf[o] = make_float2((float)v.x, (float)v.y);
        }
#undef MAT
}

// ---------------------------------------------------------------------------
// K3: relax every block of one colour.  One 512-thread workgroup per block,
// eight lanes per grid point (a residual item (point, component) per lane):
//   1. issue the block's global loads before consuming any of them (the
//      eigenvectors, eigenvalues and time factor first, then own coefficients,
//      halo neighbours outside the block, right-hand sides, lambda, V0), so one
//      memory latency covers the block;
//   2. local residual r_U = (b - K x)_U from LDS and registers (FP64), and the
//      right-hand side of the reduced block system (dc_0 eliminated by each
//      point's continuity row);
//   3. delta = V (M_r(e_k)^{-1} (V^T r)) per mode k   [K_UU^{-1} r in factored
//      form]: V^T r, the per-mode solve E3 (I - e diag(lam))^{-1} E1 chained in
//      the registers of one wave per 16 modes, then V (.) on the matrix cores;
//   4. write c_U += delta_c, lambda_U += delta_lambda;
//   5. (field steps) the new local residual is the frozen field's defect of
//      delta, point by point; repeat 3 and 4 until the block's residual fell by
//      the solver's inner tolerance (default 1e-2; 1e-13 for an exact solve) or
//      stops improving, at most n_inner times.
// BT is the precision of the factors and of step 3 (double, or float for the
// mixed path); the state and the residual of step 2 are always FP64.
// ---------------------------------------------------------------------------

// In-block neighbour of local point l in direction dir (axis dir/2, upwards if
// dir is odd) from its 2-bit code: 0 none, 1 the plain step, 2 the wrap of a
// block that spans a periodic axis; -1 when there is none.
__device__ __forceinline__ int code_nb(const LevelGeom& g, int lcode, int l, int dir) {
    const int ax = dir >> 1;
    const bool up = dir & 1;
    const int lstr = ax == 0 ? g.bdim[1] * g.bdim[2] : (ax == 1 ? g.bdim[2] : 1);
    const int code = (lcode >> (2 * dir)) & 3;
    const int step = up ? lstr : -lstr;
    const int wrap = (up ? -1 : 1) * (g.bdim[ax] - 1) * lstr;
    return code == 0 ? -1 : l + (code == 1 ? step : wrap);
}

// 1/d for normal, finite d: the hardware reciprocal estimate refined by
// Newton-Raphson steps r <- r (2 - d r), each of which squares the relative
// error (two steps in FP64, one in FP32 reach the last bit), without the
// special-case handling of a full IEEE division.
__device__ __forceinline__ double recip(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = r * (2.0 - d * r);
    return r * (2.0 - d * r);
}
__device__ __forceinline__ float recip(float d) {
    const float r = __builtin_amdgcn_rcpf(d);
    return r * (2.0f - d * r);
}

// The per-mode half of the shared-factor block solve, chained in the registers
// of one wave (no LDS round trip, no workgroup barrier): wave w (< 4) owns
// modes 16w .. 16w+15 and all nc <= 16 real columns of the reduced system.
//   X^T = R^T V            (comps x modes; A = R^T from LDS, B = V from LDS)
//   Y   = E1 X^T           (A = E1; B = X^T straight from the result registers)
//   S   = (I - e diag(lam))^{-1} Y   (per mode e, per component lam)
//   Z^T = E3 S             (A = E3; B = S from registers)
// and Z is stored [mode][ld].  A 16x16 result leaves slot r of lane
// (j + 16 q) holding row q + 4r (FP64) or 4q + r (FP32) of column j; step s of
// a 16x16x4 product takes B[k][j] from lane j + 16 kq, so the K index of
// (step s, lane group kq) is 4s + kq (FP64) or 4kq + s (FP32) and the A operand
// (E) is read in that order.  Rows or columns past nc, and modes past b, are
// masked or never stored.
template <typename T, int LD, int NCOL>
__device__ __forceinline__ void mode_chain(const T* __restrict__ Vs, const T* __restrict__ R, int b,
                                           const T* __restrict__ E1, const T* __restrict__ E3,
                                           const T* __restrict__ es, const cx<T>* __restrict__ lamv,
                                           T* __restrict__ Z, int lane, int wave) {
    constexpr int ld = LD, nc = NCOL;
    using acc_t = typename Mfma<T>::acc_t;
    constexpr bool f64 = sizeof(T) == 8;
    if (wave >= 4 || 16 * wave >= b) return;
    const int j = lane & 15, kq = lane >> 4;
    const int mode = 16 * wave + j;
    // 1. X^T = R^T V over the block's points
    acc_t x;
    for (int r = 0; r < 4; ++r) x[r] = (T)0;
    const T fc = j < nc ? (T)1 : (T)0;
    const int jc = j < nc ? j : nc - 1;
    if (b == kMaxB) {
        // one base address per operand, steps at compile-time offsets (folded into
        // the LDS instructions, so no per-step address registers); step st takes
        // point p = 16 kq + st from lane group kq (V rows 16 apart: distinct banks)
        const T* rb = R + 16 * kq * ld + jc;
        const T* vb = Vs + 16 * kq * kLdsPad + mode;
#pragma unroll
        for (int st = 0; st < kMaxB / 4; ++st) x = Mfma<T>::step(rb[st * ld] * fc, vb[st * kLdsPad], x);
    } else {
        for (int st = 0; 4 * st < b; ++st) {
            const int p = 4 * st + kq;
            const T fp = p < b ? fc : (T)0;
            const int pc = p < b ? p : b - 1;
            x = Mfma<T>::step(R[pc * ld + jc] * fp, Vs[pc * kLdsPad + mode], x);
        }
    }
    // A operand of the two mixes: E[row j][k(st, kq)], zero outside nc x nc
    auto e_at = [&](const T* E, int st) {
        const int k = f64 ? 4 * st + kq : 4 * kq + st;
        const bool in = j < nc && k < nc;
        return in ? E[jc * nc + (k < nc ? k : nc - 1)] : (T)0;
    };
    // 2. Y = E1 X^T
    acc_t y;
    for (int r = 0; r < 4; ++r) y[r] = (T)0;
#pragma unroll
    for (int st = 0; st < 4; ++st) y = Mfma<T>::step(e_at(E1, st), x[st], y);
    // 3. scaling by 1 / (1 - e lam_p) of complex entries (re, im rows 2p, 2p + 1)
    const T ev = es[mode < b ? mode : b - 1];
    acc_t sv;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = Mfma<T>::row(lane, r);
        T par;
        if constexpr (f64) par = __shfl_xor(y[r], 16);   // row ^ 1 sits 16 lanes over
        else par = y[r ^ 1];                              // row ^ 1 is the neighbouring slot
        const bool im = row & 1;
        const int pp = row >> 1;
        const cx<T> lp = lamv[pp < (nc >> 1) ? pp : (nc >> 1) - 1];
        const T xr = im ? par : y[r], xi = im ? y[r] : par;
        const T dr = (T)1 - ev * lp.r, di = -ev * lp.i;   // 1 - e lam
        const T sc = recip(dr * dr + di * di);
        sv[r] = (im ? xi * dr - xr * di : xr * dr + xi * di) * sc * (row < nc ? (T)1 : (T)0);
    }
    // 4. Z^T = E3 S
    acc_t z;
    for (int r = 0; r < 4; ++r) z[r] = (T)0;
#pragma unroll
    for (int st = 0; st < 4; ++st) z = Mfma<T>::step(e_at(E3, st), sv[st], z);
    if (mode < b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = Mfma<T>::row(lane, r);
            if (row < nc) Z[mode * ld + row] = z[r];
        }
    }
}

// Waves per SIMD the sweep is compiled for: the shared-factor variants fit 128
// registers, so two workgroups share a compute unit (LDS: under 80 KB each);
// the stored-inverse variants take 256.
template <typename BT, bool STORED>
constexpr int sweep_waves_per_simd() { return STORED ? 2 : 4; }

template <int NT, typename BT, bool STORED>
__global__ __launch_bounds__(kSweepThreads, (sweep_waves_per_simd<BT, STORED>())) void k_sweep(SweepArgs a, TimeOps<NT> to) {
    // a finished coarsest-level solve: the rest of its launches do nothing
    if (a.skip && *a.skip) return;
    constexpr int NQ = NT + 1;
    constexpr int N2 = 2 * NQ;                               // reals per point / mode
    constexpr int VPT = kMaxB * kMaxB / kSweepThreads;       // eigenvector entries per thread
    // shared factor: the block systems with dc_0 eliminated have NT unknowns per
    // mode (dlam, dc_1 .. dc_{NT-1}), so the eigenbasis transforms take NC = 2 NT
    // real columns; the stored inverses act on all NQ components
    constexpr int NC = STORED ? N2 : 2 * NT;
    constexpr int TFR = tf_record_reals(NT);                 // reals of the two mixing matrices and lam
    constexpr int TPT = (TFR + kSweepThreads - 1) / kSweepThreads;
    using C = cx<BT>;
    __shared__ BT Vs[kMaxB * kLdsPad];
    __shared__ double2 cs[kMaxB * NT];
    __shared__ double2 ls[kMaxB];
    __shared__ double v0s[kMaxB];
    __shared__ double zs[kMaxB];
    __shared__ C rs[kMaxB * NQ];   // local residual
    __shared__ C rh[kMaxB * NQ];   // per-mode solutions (stored path: V^T r first)
    __shared__ C xb[kMaxB * NQ];   // reduced right-hand side (shared factor), then the correction V y
    __shared__ BT tfs[TFR];        // shared time factor of this direction: E1, E3 real forms, lam
    __shared__ BT es[kMaxB];
    __shared__ double2 sgs[kMaxB];  // constraint residual per point (shared factor)
    __shared__ double tos[NT + NT * NT];   // the time operators U, W (indexed per lane, so staged here)
    __shared__ double2 red2[kSweepThreads / 64];   // per wave: a pass's residual norm and the initial one

    {
        // touch every 64-byte line of the sweep arguments at once, so that the later
        // reads of single arguments hit the scalar cache instead of waiting one by one
        // (the time operators that follow them are needed later, and only in part)
        const auto* kp = (const __attribute__((address_space(4))) int*)__builtin_amdgcn_kernarg_segment_ptr();
        constexpr int kEnd = (int)sizeof(SweepArgs);
        int t = kp[kEnd / 4 - 1];
#pragma unroll
        for (int off = 0; off < kEnd; off += 64) t ^= kp[off / 4];
        asm volatile("" ::"s"(t));
    }
    const LevelGeom& g = a.g;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // block of this workgroup: the colour's blocks in C order.  Everything the
    // arithmetic enumeration needs is read up front (no load depends on another).
    const int dim = g.dim, colour = a.colour, half = a.half_last, nb1 = g.nblk[1], nb2 = g.nblk[2];
    // each line along the last block axis holds nblk/2 blocks of each colour, at
    // 2i + (colour + sum of the line's other coordinates) mod 2 (computed before the
    // branch so that its inputs are loaded with the first batch)
    const int idx = (int)blockIdx.x;
    const int line = idx / half, i = idx - line * half;
    const int lead0 = dim == 3 ? line / nb1 : line;
    const int lead1 = dim == 3 ? line - lead0 * nb1 : 0;
    const int last = 2 * i + ((colour + lead0 + lead1) & 1);
    I3 bc{dim == 1 ? last : lead0, dim == 2 ? last : (dim == 3 ? lead1 : 0), dim == 3 ? last : 0};
    int blk = (bc.x * nb1 + bc.y) * nb2 + bc.z;
    if (!a.arith_blocks) {
        blk = a.blocks[idx];
        bc = block_coords(g, blk);
    }
    const int b = g.bpts;
    const int nd = 2 * g.dim;
    constexpr bool shared_tf = !STORED;
    // inner passes stop once the block's own residual fell by the solver's factor (in
    // norm), or once a pass gains less than a factor 4 (the corrections have reached
    // their rounding floor)
    const double inner_tol2 = a.inner_tol2;
    double rprev = 0.0;

    // ---- 1. the block's eigenvectors and time factor record first: they depend on
    //      the block id only, so their loads overlap the index arithmetic below.  The
    //      record is its slab's (blocks along the field axis share one): the factor of
    //      the block system with the field's time matrix taken at the dipole
    //      coordinate zf of the record ----
    const BT* tfg = static_cast<const BT*>(a.tf) + (size_t)comp(bc, g.fax) * a.tf_stride;
    const double zf = (double)tfg[TFR];
    const int iw = tid - NT;
    const double tov = tid < NT ? to.U[tid] : to.W[(iw >= 0 && iw < NT * NT) ? iw : 0];
    BT vr[VPT];
    {
        const BT* Vg = static_cast<const BT*>(a.V) + (size_t)blk * b * b;
        const int bb = b * b;
        if (b == kMaxB) {
            // full blocks: every entry in range (one base address, constant offsets)
#pragma unroll
            for (int r = 0; r < VPT; ++r) vr[r] = Vg[tid + r * kSweepThreads];
        } else {
#pragma unroll
            for (int r = 0; r < VPT; ++r) {
                const int t = tid + r * kSweepThreads;
                vr[r] = Vg[t < bb ? t : bb - 1];
            }
        }
    }
    BT tr[TPT];
    BT ep = (BT)0;
    if constexpr (shared_tf) {
#pragma unroll
        for (int r = 0; r < TPT; ++r) {
            const int t = tid + r * kSweepThreads;
            tr[r] = tfg[t < TFR ? t : TFR - 1];
        }
        ep = (BT)a.e[(size_t)blk * b + (tid < b ? tid : 0)];
    }

    // ---- 1a. addresses (no loads yet); thread = residual item (point l, component m):
    //      eight lanes per point whatever NT is (lanes m >= NT idle), so that a point's
    //      items are an aligned lane group inside one wave ----
    constexpr int LPP = 8;
    static_assert(kMaxNT <= LPP && kMaxB * LPP <= kSweepThreads, "one residual item per thread");
    const bool item = (tid & (LPP - 1)) < NT && (tid / LPP) < b;
    const int l_it = item ? tid / LPP : 0, m_it = item ? (tid & (LPP - 1)) : 0;
    const I3 lc_it = local_coords(g, l_it);
    const I3 gi_it = global_of_local(g, bc, lc_it);
    const int gj_it = point_index(g, gi_it);
    // halo neighbours (outside the block; clamped to the point itself when absent)
    // and in-block neighbours (local index, or -1), with selects only
    int hidx[6], hmask = 0, lcode = 0;
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) {
        const int ax = dir >> 1;
        const bool up = dir & 1;
        const int la = comp(lc_it, ax), ga = comp(gi_it, ax);
        const int bd = g.bdim[ax], na = g.n[ax];
        const int lstr = ax == 0 ? g.bdim[1] * g.bdim[2] : (ax == 1 ? g.bdim[2] : 1);
        const int gstr = ax == 0 ? g.n[1] * g.n[2] : (ax == 1 ? g.n[2] : 1);
        const bool used = dir < nd;
        const bool inside = up ? la + 1 < bd : la > 0;           // neighbour inside the block
        const bool self_wrap = g.periodic && g.nblk[ax] == 1;    // the block spans a periodic axis
        const bool edge = up ? ga + 1 >= na : ga == 0;           // neighbour outside the grid
        const int lstep = up ? lstr : -lstr, gstep = up ? gstr : -gstr;
        // in-block: plain step (code 1), or the wrap of a block that spans a periodic axis (code 2)
        (void)lstep;
        lcode |= (!used ? 0 : (inside ? 1 : (self_wrap ? 2 : 0))) << (2 * dir);
        // halo: plain step, or the wrap of a periodic grid; none on a Dirichlet edge
        const bool halo = used && !inside && !self_wrap && (!edge || g.periodic);
        const int hw = edge ? gj_it - (up ? 1 : -1) * (na - 1) * gstr : gj_it + gstep;
        hidx[dir] = halo ? hw : gj_it;
        hmask |= (halo ? 1 : 0) << dir;
    }
    const int tp = tid < b ? tid : 0;
    const I3 gip = global_of_local(g, bc, local_coords(g, tp));
    const int gjp = point_index(g, gip);

    // ---- 1b. loads, all in flight together ----
    const double2 own = a.c[(size_t)gj_it * NT + m_it];
    double2 hv[6];
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) hv[dir] = a.c[(size_t)hidx[dir] * NT + m_it];
    // optional right-hand sides: always one load (from the state where a side is
    // absent) times 0 or 1, so that no branch makes the loads in flight drain first
    const double2* rbp = a.bc ? a.bc + (size_t)gj_it * NT + m_it : (a.bg ? a.bg + gj_it : a.c + (size_t)gj_it * NT + m_it);
    const double2 rhsv = scl2((a.bc || a.bg) ? 1.0 : 0.0, *rbp);
    const double v0p = a.v0[gjp];
    const double2 lp = a.lam[gjp];
    const double2 sgv = scl2((a.bs && m_it == 0) ? 1.0 : 0.0, (a.bs ? a.bs : a.lam)[gj_it]);
    // ---- 1c. consume into LDS ----
    if (tid < NT + NT * NT) tos[tid] = tov;
    // a point's items are one aligned group of LPP lanes: its constraint residual
    // sigma = bs - sum_n s_n c_n is a group sum
    if constexpr (shared_tf) {
        const double sm = item ? ((m_it & 1) ? -1.0 : 1.0) : 0.0;
        const double sr = group_sum<LPP>(sm * own.x), si = group_sum<LPP>(sm * own.y);
        if (item && m_it == 0) sgs[l_it] = make_double2(sgv.x - sr, sgv.y - si);
    }
    double2 halo = make_double2(0.0, 0.0);
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) halo = add2(halo, scl2((hmask >> dir) & 1 ? 1.0 : 0.0, hv[dir]));
    if (item) cs[l_it * NT + m_it] = own;
    if (tid < b) {
        v0s[tid] = v0p;
        ls[tid] = lp;
        zs[tid] = zcoord(g, gip);
        es[tid] = ep;
    }
    if (b == kMaxB) {
        // row tid / 64 + 8 r, column tid % 64
        BT* vrow = Vs + (tid >> 6) * kLdsPad + (tid & 63);
#pragma unroll
        for (int r = 0; r < VPT; ++r) vrow[r * (kSweepThreads / 64) * kLdsPad] = vr[r];
    } else {
        const int bb = b * b;
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            const int t = tid + r * kSweepThreads;
            if (t < bb) {
                const int j = qdiv_small(t, g.rbp), k = t - j * b;
                Vs[j * kLdsPad + k] = vr[r];
            }
        }
    }
    if constexpr (shared_tf) {
#pragma unroll
        for (int r = 0; r < TPT; ++r) {
            const int t = tid + r * kSweepThreads;
            if (t < TFR) tfs[t] = tr[r];
        }
    }
    __syncthreads();

    // ---- 2. local residual (FP64); the item (l, 0) also takes the constraint row of point l ----
    double rloc = 0.0;   // squared local residual of this lane's rows (as stored)
    if (item) {
        const int l = l_it, m = m_it;
        double2 lap = add2(scl2(-2.0 * g.dim, own), halo);
#pragma unroll
        for (int dir = 0; dir < 6; ++dir) {
            const int ln = code_nb(g, lcode, l, dir);
            lap = add2(lap, scl2(ln >= 0 ? 1.0 : 0.0, cs[(ln >= 0 ? ln : l) * NT + m]));
        }
        const double2 hc = add2(scl2(-g.kin, lap), scl2(v0s[l], own));
        // time coupling: i (Q^T c)_m, with Q_nm = 2 for n > m, n - m odd (adjoint: the transpose)
        double2 tq = make_double2(0.0, 0.0);
        double2 wc = make_double2(0.0, 0.0);
        double2 sgl = sgv;
        if (STORED || a.field_on) {
            // every component: the field's W row, and (stored path) the constraint row
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const double2 cn = cs[l * NT + n];
                const bool cpl = a.adjoint ? (n < m && ((m - n) & 1)) : (n > m && ((n - m) & 1));
                tq = add2(tq, scl2(cpl ? 1.0 : 0.0, cn));
                if (a.field_on) wc = add2(wc, scl2(tos[NT + m * NT + n], cn));
                sgl = (n & 1) ? add2(sgl, cn) : sub2(sgl, cn);
            }
        } else {
            // only the coupled components m + 1, m + 3, ... (adjoint m - 1, m - 3, ...)
#pragma unroll
            for (int k = 0; k < (NT + 1) / 2; ++k) {
                const int n = a.adjoint ? m - 1 - 2 * k : m + 1 + 2 * k;
                const bool in = n >= 0 && n < NT;
                tq = add2(tq, scl2(in ? 1.0 : 0.0, cs[l * NT + (in ? n : m)]));
            }
        }
        const double2 tim = a.adjoint ? make_double2(2.0 * tq.y, -2.0 * tq.x) : make_double2(-2.0 * tq.y, 2.0 * tq.x);
        const double sm = (m & 1) ? -1.0 : 1.0;
        double2 row = sub2(sub2(tim, scl2(tos[m], hc)), scl2(zs[l], wc));
        row = add2(row, scl2(sm, ls[l]));
        const double2 rho = sub2(rhsv, row);
        const C rhof = C{(BT)rho.x, (BT)rho.y};
        rs[l * NQ + m] = rhof;
        rloc = (double)rhof.r * rhof.r + (double)rhof.i * rhof.i;
        if (m == 0) {
            if constexpr (shared_tf) sgl = sgs[l];   // the same rounding as the reduced system
            const C sgf = C{(BT)sgl.x, (BT)sgl.y};
            rs[l * NQ + NT] = sgf;
            rloc += (double)sgf.r * sgf.r + (double)sgf.i * sgf.i;
        }
        if constexpr (shared_tf) {
            // right-hand side of the reduced system (dc_0 eliminated): rho - sigma K(e) e_0
            // with K(e) = (time coupling) - e U - zf W, i.e. + U_0 (A sigma) on component 0
            // (A: the block operator, whose eigenvalues are e; sigma of the in-block
            // neighbours from sgs), + zf W_m0 sigma on every component and, adjoint,
            // + 2 i sigma on odd components
            double2 r = rho;
            const double2 sg = sgs[l];
            if (m == 0) {
                double2 lin = make_double2(0.0, 0.0);
#pragma unroll
                for (int dir = 0; dir < 6; ++dir) {
                    const int ln = code_nb(g, lcode, l, dir);
                    lin = add2(lin, scl2(ln >= 0 ? 1.0 : 0.0, sgs[ln >= 0 ? ln : l]));
                }
                const double2 asg = add2(scl2(g.kin, sub2(scl2(2.0 * g.dim, sg), lin)), scl2(v0s[l], sg));
                r = add2(r, scl2(tos[0], asg));
            }
            if (a.field_on) r = add2(r, scl2(zf * tos[NT + m * NT], sg));
            if (a.adjoint && (m & 1)) r = add2(r, make_double2(-2.0 * sg.y, 2.0 * sg.x));
            xb[l * NQ + m] = C{(BT)r.x, (BT)r.y};
        }
    }
    __syncthreads();
    double r0n = 0.0;

    const C* Mi = static_cast<const C*>(a.Minv);
    for (int pass = 0; pass <= a.n_inner; ++pass) {
        if constexpr (STORED) {
            // ---- 3a. rh[k][.] = sum_j V[j][k] rs[j][.]  (matrix cores) ----
            {
                const auto acc = tile_gemm<BT, true, NC, N2>(Vs, reinterpret_cast<const BT*>(rs), b, lane, wave);
                tile_store<BT>(reinterpret_cast<BT*>(rh), b, NC, N2, lane, wave, acc);
            }
            __syncthreads();
            // ---- 3b. per-mode time solve ----
            // stored inverses M(e_k)^{-1}; waves 0..3, thread (k, pg) computes rows pg, pg+4, pg+8
            const int k = tid & 63, pg = tid >> 6;
            const bool act = pg < 4;
            C out[3];
            if (act && k < b) {
                C rv[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) rv[q] = rh[k * NQ + q];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const int p = pg + 4 * r;
                    C acc = C{0, 0};
                    if (p < NQ) {
#pragma unroll
                        for (int q = 0; q < NQ; ++q) {
                            if (!a.adjoint) {
                                const C mv = Mi[(((size_t)blk * NQ + p) * NQ + q) * b + k];
                                acc = acc + cmul(mv, rv[q]);
                            } else {
                                const C mv = Mi[(((size_t)blk * NQ + q) * NQ + p) * b + k];
                                acc = acc + cmulc(mv, rv[q]);
                            }
                        }
                    }
                    out[r] = acc;
                }
            }
            __syncthreads();
            if (act && k < b) {
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    const int p = pg + 4 * r;
                    if (p < NQ) rh[k * NQ + p] = out[r];
                }
            }
        } else {
            // ---- 3a + 3b. into the block eigenbasis and the per-mode solve
            //      M_r(e)^{-1} = E3 (I - e diag(lam))^{-1} E1, chained per wave ----
            const BT* E1 = tfs;
            const BT* E3 = tfs + 4 * NT * NT;
            const C* lamv = reinterpret_cast<const C*>(tfs + 8 * NT * NT);
            mode_chain<BT, N2, NC>(Vs, reinterpret_cast<const BT*>(xb), b, E1, E3, es, lamv,
                                   reinterpret_cast<BT*>(rh), lane, wave);
        }
        __syncthreads();
        // ---- 3c. back to points: xb[j][.] = sum_k V[j][k] rh[k][.] ----
        {
            const auto acc = tile_gemm<BT, false, NC, N2>(Vs, reinterpret_cast<const BT*>(rh), b, lane, wave);
            tile_store<BT>(reinterpret_cast<BT*>(xb), b, NC, N2, lane, wave, acc);
        }
        __syncthreads();
        // ---- 4. corrections of this thread's item (point l, component m) and, for
        //      m = 0, of the multiplier of point l.  Shared factor: xb[l] holds
        //      (dlam, dc_1 .. dc_{NT-1}) and dc_0 = sigma - sum_{j>=1} s_j dc_j ----
        const bool last = pass == a.n_inner;
        C dv = C{0, 0}, dl = C{0, 0};
        if constexpr (STORED) {
            if (item) {
                dv = xb[l_it * NQ + m_it];
                dl = xb[l_it * NQ + NT];
            }
        } else {
            // every lane reads its own entry; dc_0 from a group sum (all lanes active)
            const C x = xb[l_it * NQ + m_it];
            const BT sm = (!item || m_it == 0) ? (BT)0 : ((m_it & 1) ? (BT)-1 : (BT)1);
            const BT sr = group_sum<LPP>(sm * x.r), si = group_sum<LPP>(sm * x.i);
            if (m_it > 0) {
                dv = x;
            } else {
                const C sg = rs[l_it * NQ + NT];
                dv = C{sg.r - sr, sg.i - si};
                dl = x;
            }
        }
        // the updated state goes straight to HBM, before the pass check: the block
        // owns its points during the launch, so when another pass follows its
        // result simply overwrites this one
        if (item) {
            const int l = l_it, m = m_it;
            a.c[(size_t)gj_it * NT + m] = add2(cs[l * NT + m], make_double2((double)dv.r, (double)dv.i));
            if (m == 0) a.lam[gj_it] = add2(ls[l], make_double2((double)dl.r, (double)dl.i));
        }
        if (last) {
            // the cap was reached: with a field the last correction is left unchecked
            if (a.passes && tid == 0)
                a.passes[blk] = (unsigned char)(pass | ((a.n_inner > 0 && a.field_on) ? 0x80 : 0));
            break;
        }
        // inner pass: keep the state in LDS.  The correction solved the block system
        // with the field taken at zf exactly, so the new local residual r - K_bb delta
        // is the rest of the field's term on this point alone:
        //   row (l, m):  (z_l - zf) (W delta_l)_m,   constraint row: 0
        // (written in place: no neighbour's correction is needed).  The reduced
        // right-hand side of the next pass is that residual itself (sigma = 0).
        if (item) {
            const int l = l_it, m = m_it;
            cs[l * NT + m] = add2(cs[l * NT + m], make_double2((double)dv.r, (double)dv.i));
            if (m == 0) ls[l] = add2(ls[l], make_double2((double)dl.r, (double)dl.i));
            rh[l * NQ + m] = dv;   // this point's corrections, for its lane group
        }
        // a point's lanes are one group inside a wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        double loc = 0.0;
        if (item) {
            const int l = l_it, m = m_it;
            C wd = C{0, 0};
            if (a.field_on) {
#pragma unroll 1
                for (int n = 0; n < NT; ++n) wd = wd + rmul((BT)tos[NT + m * NT + n], rh[l * NQ + n]);
            }
            const C rn = rmul((BT)(zs[l] - zf), wd);
            rs[l * NQ + m] = rn;
            if (m == 0) rs[l * NQ + NT] = C{0, 0};
            if constexpr (shared_tf) xb[l * NQ + m] = rn;
            loc = (double)rn.r * rn.r + (double)rn.i * rn.i;
        }
        {
            // stop the defect corrections once the local system is solved: the wave
            // partials of this pass's norm (and, on the first pass, of the initial
            // one) summed by every thread after one barrier, the same in every lane
            const double ws = wave_total(loc), w0 = pass == 0 ? wave_total(rloc) : 0.0;
            if (lane == 0) red2[wave] = make_double2(ws, w0);
            __syncthreads();
            double rn = 0.0, r0t = 0.0;
#pragma unroll
            for (int w = 0; w < kSweepThreads / 64; ++w) {
                const double2 v = red2[w];
                rn += v.x;
                r0t += v.y;
            }
            if (pass == 0) r0n = r0t;
            const bool solved = __builtin_amdgcn_readfirstlane(rn <= inner_tol2 * r0n ? 1 : 0) != 0;
            const bool done =
                solved || __builtin_amdgcn_readfirstlane(rn > 0.0625 * (pass > 0 ? rprev : r0n) ? 1 : 0) != 0;
            rprev = rn;
            if (done) {
                if (a.passes && tid == 0) a.passes[blk] = (unsigned char)(pass | (solved ? 0 : 0x80));
                break;
            }
        }
    }
}

// The FP32 shared-factor colour sweep with two time components per lane: four
// lanes per point (lane q of a point takes m = q and m = q + 4), so a 64-point
// block is one wave per SIMD.  The per-point index arithmetic is done once for
// two components, every wave takes part in the matrix-core steps, and with a
// block geometry fixed at compile time (up to 128 registers and under 40 KB of
// LDS) four blocks share a compute unit, otherwise three (the general geometry
// takes up to 168).  The arithmetic of each item is that of k_sweep<NT, float,
// false>.  GEO: 3 = a 3D level with 4 x 4 x 4 blocks, 2 = a 2D level with 8 x 8
// blocks, both known at compile time (the block geometry's divisions become
// shifts and its tests constants); 0 = the level's block geometry.
template <int NT, int GEO>
__global__ __launch_bounds__(kPairThreads, GEO != 0 ? 4 : 3) void k_sweep_pair(SweepArgs a, TimeOps<NT> to) {
    using BT = float;
    using C = cx<BT>;
    // a finished coarsest-level solve: the rest of its launches do nothing
    if (a.skip && *a.skip) return;
    constexpr int THR = kPairThreads;
    constexpr int NW = THR / 64;                             // waves per block
    constexpr int NQ = NT + 1;
    constexpr int N2 = 2 * NQ;                               // reals per point / mode
    constexpr int NC = 2 * NT;                               // real columns of the reduced system
    constexpr int VPT = kMaxB * kMaxB / THR;                 // eigenvector entries per thread
    constexpr int TFR = tf_record_reals(NT);                 // reals of the two mixing matrices and lam
    constexpr int TPT = (TFR + THR - 1) / THR;
    constexpr int LPP = 4, IPL = 2;                          // lanes per point, items per lane
    static_assert(kMaxNT <= LPP * IPL && kMaxB * LPP == THR && NW == 4, "every residual item has a lane");
    __shared__ BT Vs[kMaxB * kLdsPad];
    __shared__ double2 cs[(kMaxB + 1) * NT];   // row kMaxB: zeros (absent neighbours); layout csx
    // Slot of (point l, component m) in cs: with N_t = 8 the components of row l are
    // permuted by (l / 2) mod 8, so that both the 64 lanes reading one component of
    // 16 points and the 16 point groups reading one component each spread over all
    // LDS banks (128-byte rows would otherwise meet in two bank groups).
    auto csx = [](int l, int m) { return l * NT + (NT == 8 ? m ^ ((l >> 1) & 7) : m); };
    __shared__ double2 ls[kMaxB];
    __shared__ C sgr[kMaxB];       // constraint residual of each point
    __shared__ C rh[kMaxB * NQ];   // per-mode solutions
    __shared__ C xb[kMaxB * NQ];   // reduced right-hand side, then the correction V y
    __shared__ BT tfs[TFR];        // shared time factor of this direction: E1, E3 real forms, lam
    __shared__ BT es[kMaxB];
    __shared__ double2 sgs[kMaxB + 1];  // constraint residual per point (row kMaxB: zero)
    __shared__ double tos[NT];             // the time operator U (indexed per lane, so staged here)
    __shared__ double2 tcs[NT * NT];       // at n NT + m: W_mn and the 0/1 pattern of the Q coupling
    __shared__ double2 red2[NW];    // per wave: the bound of an inner pass's residual norm and the initial one
    __shared__ double red3[NW];     // per wave: an inner pass's residual norm

    {
        // touch every 64-byte line of the sweep arguments at once (see k_sweep)
        const auto* kp = (const __attribute__((address_space(4))) int*)__builtin_amdgcn_kernarg_segment_ptr();
        constexpr int kEnd = (int)sizeof(SweepArgs);
        int t = kp[kEnd / 4 - 1];
#pragma unroll
        for (int off = 0; off < kEnd; off += 64) t ^= kp[off / 4];
        asm volatile("" ::"s"(t));
    }
    const LevelGeom& g = a.g;
    // the block geometry (compile-time when FIX): rank, extents, local
    // coordinates of block point l, global coordinates
    constexpr bool FIX = GEO != 0;
    constexpr int FE = GEO == 3 ? 4 : 8;   // extent per used axis of a fixed geometry
    const int gdim = FIX ? GEO : g.dim;
    auto bdim = [&](int ax) { return FIX ? (ax < GEO ? FE : 1) : g.bdim[ax]; };
    auto local_of = [&](int l) {
        if constexpr (GEO == 3) return I3{l >> 4, (l >> 2) & 3, l & 3};
        else if constexpr (GEO == 2) return I3{l >> 3, l & 7, 0};
        else return local_coords(g, l);
    };
    auto global_of = [&](const I3& blk3, const I3& lc) {
        return I3{blk3.x * bdim(0) + lc.x, blk3.y * bdim(1) + lc.y, blk3.z * bdim(2) + lc.z};
    };
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // block of this workgroup (as in k_sweep)
    const int dim = gdim, colour = a.colour, half = a.half_last, nb1 = g.nblk[1], nb2 = g.nblk[2];
    const int idx = (int)blockIdx.x;
    const int line = idx / half, i = idx - line * half;
    const int lead0 = dim == 3 ? line / nb1 : line;
    const int lead1 = dim == 3 ? line - lead0 * nb1 : 0;
    const int last = 2 * i + ((colour + lead0 + lead1) & 1);
    I3 bc{dim == 1 ? last : lead0, dim == 2 ? last : (dim == 3 ? lead1 : 0), dim == 3 ? last : 0};
    int blk = (bc.x * nb1 + bc.y) * nb2 + bc.z;
    if (!a.arith_blocks) {
        blk = a.blocks[idx];
        bc = block_coords(g, blk);
    }
    const int b = FIX ? 64 : g.bpts;
    const int nd = 2 * gdim;
    const double inner_tol2 = a.inner_tol2;   // inner passes: see k_sweep
    double rprev = 0.0;

    // ---- 1. eigenvectors and the slab's time factor record (see k_sweep) ----
    const BT* tfg = static_cast<const BT*>(a.tf) + (size_t)comp(bc, g.fax) * a.tf_stride;
    const double zf = (double)tfg[TFR];
    const int iw = tid - NT;
    const double tov = tid < NT ? to.U[tid] : to.W[(iw >= 0 && iw < NT * NT) ? iw : 0];
    BT vr[VPT];
    {
        const BT* Vg = static_cast<const BT*>(a.V) + (size_t)blk * b * b;
        const int bb = b * b;
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            // FIX: b = 64, every entry in range (one base address, constant offsets)
            const int t = tid + r * THR;
            vr[r] = Vg[FIX ? t : (t < bb ? t : bb - 1)];
        }
    }
    BT tr[TPT];
#pragma unroll
    for (int r = 0; r < TPT; ++r) {
        const int t = tid + r * THR;
        tr[r] = tfg[t < TFR ? t : TFR - 1];
    }
    const BT ep = (BT)a.e[(size_t)blk * b + (tid < b ? tid : 0)];

    // ---- 1a. addresses: thread = point l = tid / 4 and the items (l, q), (l, q + 4)
    //      (q = tid % 4; items past NT or the block are idle and load a clamped,
    //      valid address) ----
    const int l_it = tid / LPP < b ? tid / LPP : 0;
    const int q_it = tid & (LPP - 1);
    bool item[IPL];
    int m_it[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        item[k] = q_it + LPP * k < NT && tid / LPP < b;
        m_it[k] = item[k] ? q_it + LPP * k : 0;
    }
    const I3 lc_it = local_of(l_it);
    const I3 gi_it = global_of(bc, lc_it);
    const int gj_it = point_index(g, gi_it);
    // neighbours: nrow[dir] is the in-block neighbour's row in LDS (the zero row
    // kMaxB when there is none); the halo comes from HBM, one load per direction,
    // or with FIX one per axis (a point of a 4- or 8-wide block lies on at most one
    // of the block's two faces across an axis)
    constexpr int NH = FIX ? GEO : 6;
    int hidx[NH], nrow[6], hmask = 0;
#pragma unroll
    for (int s = 0; s < NH; ++s) hidx[s] = gj_it;
    if constexpr (FIX) {
        // whether the block's low / high face across an axis has a halo, and the
        // offset to it, are the same for the whole block; a point only asks
        // whether it lies on that face
#pragma unroll
        for (int dir = 2 * GEO; dir < 6; ++dir) nrow[dir] = kMaxB;
#pragma unroll
        for (int ax = 0; ax < GEO; ++ax) {
            const int la = comp(lc_it, ax), bax = comp(bc, ax), nba = g.nblk[ax], na = g.n[ax];
            const int gstr = ax == 0 ? g.n[1] * g.n[2] : (ax == 1 ? g.n[2] : 1);
            const int lstr = GEO == 3 ? (ax == 0 ? 16 : (ax == 1 ? 4 : 1)) : (ax == 0 ? 8 : 1);
            const bool self_wrap = g.periodic && nba == 1;
            const bool lo_ok = !self_wrap && (bax > 0 || g.periodic);
            const bool hi_ok = !self_wrap && (bax < nba - 1 || g.periodic);
            const int lo_off = bax > 0 ? -gstr : (na - 1) * gstr;
            const int hi_off = bax < nba - 1 ? gstr : -(na - 1) * gstr;
            const bool at_lo = la == 0, at_hi = la == FE - 1;
            const bool halo = (at_lo && lo_ok) || (at_hi && hi_ok);
            hidx[ax] = gj_it + (halo ? (at_lo ? lo_off : hi_off) : 0);
            hmask |= (halo ? 1 : 0) << ax;
            nrow[2 * ax] = !at_lo ? l_it - lstr : (self_wrap ? l_it + (FE - 1) * lstr : kMaxB);
            nrow[2 * ax + 1] = !at_hi ? l_it + lstr : (self_wrap ? l_it - (FE - 1) * lstr : kMaxB);
        }
    } else
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) {
        const int ax = dir >> 1;
        const bool up = dir & 1;
        const int la = comp(lc_it, ax), ga = comp(gi_it, ax);
        const int bd = bdim(ax), na = g.n[ax];
        const int gstr = ax == 0 ? g.n[1] * g.n[2] : (ax == 1 ? g.n[2] : 1);
        const int lstr = ax == 0 ? bdim(1) * bdim(2) : (ax == 1 ? bdim(2) : 1);
        const bool used = dir < nd;
        const bool inside = up ? la + 1 < bd : la > 0;
        const bool self_wrap = g.periodic && g.nblk[ax] == 1;
        const bool edge = up ? ga + 1 >= na : ga == 0;
        const int gstep = up ? gstr : -gstr;
        const int lstep = inside ? (up ? lstr : -lstr) : (up ? -1 : 1) * (bd - 1) * lstr;
        nrow[dir] = used && (inside || self_wrap) ? l_it + lstep : kMaxB;
        const bool halo = used && !inside && !self_wrap && (!edge || g.periodic);
        const int hw = edge ? gj_it - (up ? 1 : -1) * (na - 1) * gstr : gj_it + gstep;
        const int s = FIX ? ax : dir;
        hidx[s] = halo ? hw : hidx[s];
        hmask |= (halo ? 1 : 0) << s;
    }
    const int tp = tid < b ? tid : 0;
    const I3 gip = global_of(bc, local_of(tp));
    const int gjp = point_index(g, gip);

    // ---- 1b. loads, all in flight together ----
    double2 own[IPL], hv[IPL][NH], rhsv[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        own[k] = a.c[(size_t)gj_it * NT + m_it[k]];
#pragma unroll
        for (int s = 0; s < NH; ++s) hv[k][s] = a.c[(size_t)hidx[s] * NT + m_it[k]];
    }
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const double2* rbp = a.bc ? a.bc + (size_t)gj_it * NT + m_it[k]
                                  : (a.bg ? a.bg + gj_it : a.c + (size_t)gj_it * NT + m_it[k]);
        rhsv[k] = scl2((a.bc || a.bg) ? 1.0 : 0.0, *rbp);
    }
    const double v0l = a.v0[gj_it];   // the point's potential (each of its lanes loads it)
    const double2 lp = a.lam[gjp];
    // the point's constraint right-hand side (lane q = 0 holds m = 0)
    const double2 sgv = scl2((a.bs && q_it == 0) ? 1.0 : 0.0, (a.bs ? a.bs : a.lam)[gj_it]);
    // ---- 1c. consume into LDS; sigma = bs - sum_n s_n c_n as a sum over the point's lanes ----
    if (tid < NT) tos[tid] = tov;
    if (iw >= 0 && iw < NT * NT) {
        const int mm = iw / NT, nn = iw - mm * NT;
        const bool cpl = a.adjoint ? (nn < mm && ((mm - nn) & 1)) : (nn > mm && ((nn - mm) & 1));
        tcs[nn * NT + mm] = make_double2(tov, cpl ? 1.0 : 0.0);
    }
    if (tid < NT) cs[kMaxB * NT + tid] = make_double2(0.0, 0.0);
    if (tid == NT) sgs[kMaxB] = make_double2(0.0, 0.0);
    {
        double pr = 0.0, pi = 0.0;
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            const double sm = item[k] ? ((m_it[k] & 1) ? -1.0 : 1.0) : 0.0;
            pr += sm * own[k].x;
            pi += sm * own[k].y;
        }
        const double sr = group_sum<LPP>(pr), si = group_sum<LPP>(pi);
        if (tid / LPP < b && q_it == 0) sgs[l_it] = make_double2(sgv.x - sr, sgv.y - si);
    }
    // the parts of (H c) at the item that need no other in-block point:
    // -kin (halo - 2 d c) + V0 c (the in-block neighbours are added from LDS)
    double2 pre[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        double2 halo = scl2(-2.0 * gdim, own[k]);
#pragma unroll
        for (int s = 0; s < NH; ++s) halo = add2(halo, scl2((hmask >> s) & 1 ? 1.0 : 0.0, hv[k][s]));
        pre[k] = add2(scl2(-g.kin, halo), scl2(v0l, own[k]));
        // formed here, so that the halo values need no registers past the barrier
        asm volatile("" : "+v"(pre[k].x), "+v"(pre[k].y));
        if (item[k]) cs[csx(l_it, m_it[k])] = own[k];
    }
    if (tid < b) {
        ls[tid] = lp;
        es[tid] = ep;
    }
    if constexpr (FIX) {
        // row tid / 64 + 4 r, column tid % 64: one base address, constant offsets
        BT* vrow = Vs + (tid >> 6) * kLdsPad + (tid & 63);
#pragma unroll
        for (int r = 0; r < VPT; ++r) vrow[r * (THR / 64) * kLdsPad] = vr[r];
    } else {
        const int bb = b * b;
#pragma unroll
        for (int r = 0; r < VPT; ++r) {
            const int t = tid + r * THR;
            if (t < bb) {
                const int j = qdiv_small(t, g.rbp), k = t - j * b;
                Vs[j * kLdsPad + k] = vr[r];
            }
        }
    }
#pragma unroll
    for (int r = 0; r < TPT; ++r) {
        const int t = tid + r * THR;
        if (t < TFR) tfs[t] = tr[r];
    }
    __syncthreads();

    // ---- 2. local residual (FP64) and the reduced right-hand side (see k_sweep) ----
    const double zl = zcoord(g, gi_it);   // the point's coordinate along the field
    double rloc = 0.0;                    // squared local residual of this lane's rows (as stored)
    // slots of the in-block neighbours' component m_it[0]; with N_t = 8 component
    // m_it[0] + 4 sits at slot ^ 4 (the row permutation changes the index by an xor)
    int nbs0[6];
#pragma unroll
    for (int dir = 0; dir < 6; ++dir) nbs0[dir] = csx(nrow[dir], m_it[0]);
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        if (!item[k]) continue;
        const int l = l_it, m = m_it[k];
        // m = m_it[0] + 4 k (with N_t <= 4 the second item is idle: its reads stay in row)
        const int sx = (k == 0 || NT != 8) ? 0 : 4;
        double2 nbs = cs[nbs0[0] ^ sx];
#pragma unroll
        for (int dir = 1; dir < 6; ++dir) nbs = add2(nbs, cs[nbs0[dir] ^ sx]);
        const double2 hc = add2(pre[k], scl2(-g.kin, nbs));
        double2 tq = make_double2(0.0, 0.0);
        double2 wc = make_double2(0.0, 0.0);
        if (a.field_on) {
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                const double2 cn = cs[csx(l, n)];
                const double2 wq = tcs[n * NT + m];
                tq = add2(tq, scl2(wq.y, cn));
                wc = add2(wc, scl2(wq.x, cn));
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < (NT + 1) / 2; ++kk) {
                const int n = a.adjoint ? m - 1 - 2 * kk : m + 1 + 2 * kk;
                const bool in = n >= 0 && n < NT;
                tq = add2(tq, scl2(in ? 1.0 : 0.0, cs[csx(l, in ? n : m)]));
            }
        }
        const double2 tim = a.adjoint ? make_double2(2.0 * tq.y, -2.0 * tq.x) : make_double2(-2.0 * tq.y, 2.0 * tq.x);
        const double sm = (m & 1) ? -1.0 : 1.0;
        double2 row = sub2(sub2(tim, scl2(tos[m], hc)), scl2(zl, wc));
        row = add2(row, scl2(sm, ls[l]));
        const double2 rho = sub2(rhsv[k], row);
        const C rhof = C{(BT)rho.x, (BT)rho.y};
        rloc += (double)rhof.r * rhof.r + (double)rhof.i * rhof.i;
        const double2 sg = sgs[l];
        if (m == 0) {
            const C sgf = C{(BT)sg.x, (BT)sg.y};
            sgr[l] = sgf;
            rloc += (double)sgf.r * sgf.r + (double)sgf.i * sgf.i;
        }
        double2 r = rho;
        if (m == 0) {
            double2 lin = make_double2(0.0, 0.0);
#pragma unroll
            for (int dir = 0; dir < 6; ++dir) lin = add2(lin, sgs[nrow[dir]]);
            const double2 asg = add2(scl2(g.kin, sub2(scl2(2.0 * gdim, sg), lin)), scl2(v0l, sg));
            r = add2(r, scl2(tos[0], asg));
        }
        if (a.field_on) r = add2(r, scl2(zf * tcs[m].x, sg));
        if (a.adjoint && (m & 1)) r = add2(r, make_double2(-2.0 * sg.y, 2.0 * sg.x));
        xb[l * NQ + m] = C{(BT)r.x, (BT)r.y};
    }
    __syncthreads();
    double r0n = 0.0;

    for (int pass = 0; pass <= a.n_inner; ++pass) {
        // ---- 3a + 3b. into the block eigenbasis and the per-mode solve, one wave per
        //      16 modes (all four waves) ----
        const BT* E1 = tfs;
        const BT* E3 = tfs + 4 * NT * NT;
        const C* lamv = reinterpret_cast<const C*>(tfs + 8 * NT * NT);
        mode_chain<BT, N2, NC>(Vs, reinterpret_cast<const BT*>(xb), b, E1, E3, es, lamv, reinterpret_cast<BT*>(rh),
                               lane, wave);
        __syncthreads();
        // ---- 3c. back to points: xb[j][.] = sum_k V[j][k] rh[k][.] (one 16-row tile per wave) ----
        {
            const auto acc = tile_gemm<BT, false, NC, N2>(Vs, reinterpret_cast<const BT*>(rh), b, lane, wave);
            tile_store<BT>(reinterpret_cast<BT*>(xb), b, NC, N2, lane, wave, acc);
        }
        __syncthreads();
        // ---- 4. corrections: xb[l] holds (dlam, dc_1 .. dc_{NT-1}), dc_0 = sigma -
        //      sum_{j>=1} s_j dc_j as a sum over the point's lanes ----
        const bool last = pass == a.n_inner;
        C dv[IPL], dl = C{0, 0};
        {
            C x[IPL];
            BT pr = (BT)0, pi = (BT)0;
#pragma unroll
            for (int k = 0; k < IPL; ++k) {
                x[k] = xb[l_it * NQ + m_it[k]];
                const BT sm = (!item[k] || m_it[k] == 0) ? (BT)0 : ((m_it[k] & 1) ? (BT)-1 : (BT)1);
                pr += sm * x[k].r;
                pi += sm * x[k].i;
            }
            const BT sr = group_sum<LPP>(pr), si = group_sum<LPP>(pi);
            const C sg = sgr[l_it];
#pragma unroll
            for (int k = 0; k < IPL; ++k) dv[k] = m_it[k] > 0 ? x[k] : C{sg.r - sr, sg.i - si};
            dl = x[0];   // used by the lane holding m = 0 only
        }
        // the updated state goes straight to HBM, before the pass check: the block
        // owns its points during the launch, so when another pass follows (rarely)
        // its result simply overwrites this one
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            if (!item[k]) continue;
            const int l = l_it, m = m_it[k];
            a.c[(size_t)gj_it * NT + m] = add2(cs[csx(l, m)], make_double2((double)dv[k].r, (double)dv[k].i));
            if (m == 0) a.lam[gj_it] = add2(ls[l], make_double2((double)dl.r, (double)dl.i));
        }
        // inner pass check (see k_sweep): the next local residual would be
        // (z_l - zf) (W delta_l)_m on row (l, m) and 0 on the constraint rows; its
        // norm against the initial one decides (uniformly: every thread sums the
        // same wave partials after one barrier) whether the block is done
        bool done = last;
        unsigned char pbyte = (unsigned char)(pass | ((a.n_inner > 0 && a.field_on) ? 0x80 : 0));
        C rn[IPL];
        if (!last) {
            // first a bound: ||(z - zf) W delta||^2 <= sum_l (z_l - zf)^2 ||W||^2 ||delta_l||^2;
            // when it already meets the tolerance the block is solved (as the exact
            // defect below would find), else the exact defect decides
            {
                double bl = 0.0;
#pragma unroll
                for (int k = 0; k < IPL; ++k)
                    if (item[k]) bl += (double)dv[k].r * dv[k].r + (double)dv[k].i * dv[k].i;
                bl *= (zl - zf) * (zl - zf);
                const double wb = wave_total(bl), w0 = pass == 0 ? wave_total(rloc) : 0.0;
                if (lane == 0) red2[wave] = make_double2(wb, w0);
                __syncthreads();
                double bt = 0.0, r0t = 0.0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    const double2 v = red2[w];
                    bt += v.x;
                    r0t += v.y;
                }
                if (pass == 0) r0n = r0t;
                if (__builtin_amdgcn_readfirstlane(a.wbound2 * bt <= inner_tol2 * r0n ? 1 : 0) != 0) {
                    if (a.passes && tid == 0) a.passes[blk] = (unsigned char)pass;
                    break;
                }
            }
            // delta of every component of the point, from the point's four lanes
            // (lane q holds components q and q + 4)
            C dn[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) dn[n] = quad_bcast(dv[n >> 2], n & 3);
            double loc = 0.0;
#pragma unroll
            for (int k = 0; k < IPL; ++k) {
                const int m = m_it[k];
                C wd = C{0, 0};
                if (a.field_on) {
#pragma unroll
                    for (int n = 0; n < NT; ++n) wd = wd + rmul((BT)tcs[n * NT + m].x, dn[n]);
                }
                rn[k] = item[k] ? rmul((BT)(zl - zf), wd) : C{0, 0};
                loc += (double)rn[k].r * rn[k].r + (double)rn[k].i * rn[k].i;
            }
            const double ws = wave_total(loc);
            if (lane == 0) red3[wave] = ws;
            __syncthreads();
            double rnt = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) rnt += red3[w];
            // the same in every lane: taken as a scalar, so the branches below are uniform
            const bool solved = __builtin_amdgcn_readfirstlane(rnt <= inner_tol2 * r0n ? 1 : 0) != 0;
            done = solved || __builtin_amdgcn_readfirstlane(rnt > 0.0625 * (pass > 0 ? rprev : r0n) ? 1 : 0) != 0;
            rprev = rnt;
            pbyte = (unsigned char)(pass | (solved ? 0 : 0x80));
        }
        if (done) {
            if (a.passes && tid == 0) a.passes[blk] = pbyte;
            break;
        }
        // another pass: the state stays in LDS and the new local residual is the
        // right-hand side
#pragma unroll
        for (int k = 0; k < IPL; ++k) {
            if (!item[k]) continue;
            const int l = l_it, m = m_it[k];
            cs[csx(l, m)] = add2(cs[csx(l, m)], make_double2((double)dv[k].r, (double)dv[k].i));
            if (m == 0) {
                ls[l] = add2(ls[l], make_double2((double)dl.r, (double)dl.i));
                sgr[l] = C{0, 0};
            }
            xb[l * NQ + m] = rn[k];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// K11: step I/O and the adjoint right-hand side.
// ---------------------------------------------------------------------------
// Initial guess c_j0 = psi_j (s_0 = T_0(t0) = 1), c_jn = 0 (n >= 1),
// lambda = 0: one thread per (point, component), so the stores of c are
// coalesced.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_init_forward(int P, const double2* __restrict__ psi,
                                                           double2* __restrict__ c, double2* __restrict__ lam,
                                                           double2* __restrict__ bs) {
    const size_t k = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= (size_t)P * NT) return;
    const size_t j = k / NT;
    const int m = (int)(k - j * NT);
    const double2 p = psi[j];
    c[k] = m == 0 ? p : make_double2(0.0, 0.0);
    if (m == 0) {
        lam[j] = make_double2(0.0, 0.0);
        bs[j] = p;
    }
}

// Zero state (the adjoint solve starts from mu = 0).
template <int NT>
__global__ __launch_bounds__(kThreads) void k_init_zero(int P, double2* __restrict__ c,
                                                        double2* __restrict__ lam) {
    // one thread per (point, component): coalesced stores of c
    const size_t k = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= (size_t)P * NT) return;
    c[k] = make_double2(0.0, 0.0);
    if (k % NT == 0) lam[k / NT] = make_double2(0.0, 0.0);
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_end_eval(int P, const double2* __restrict__ c,
                                                       double2* __restrict__ psi) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= P) return;
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int n = 0; n < NT; ++n) acc = add2(acc, c[(size_t)j * NT + n]);
    psi[j] = acc;
}

// End of one step and start of the next: psi = x(t0 + dt) as in k_end_eval
// (the components summed in the same order), and the next initial state from
// it as in k_init_forward, written to a second set of buffers (c is left as it
// is).  One thread per (point, component), so every load and store is
// coalesced; the components of a point meet in LDS.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_advance(int P, const double2* __restrict__ c,
                                                      double2* __restrict__ psi, double2* __restrict__ cn,
                                                      double2* __restrict__ lamn, double2* __restrict__ bsn) {
    constexpr int PW = kThreads / NT;  // points per workgroup
    __shared__ double2 cs[PW * NT];
    const int t = threadIdx.x;
    const int lp = t / NT, m = t - lp * NT;
    const size_t j = (size_t)blockIdx.x * PW + lp;
    const bool act = lp < PW && j < (size_t)P;
    if (act) cs[t] = c[j * NT + m];
    __syncthreads();
    if (!act) return;
    double2 ps = make_double2(0.0, 0.0);
#pragma unroll
    for (int n = 0; n < NT; ++n) ps = add2(ps, cs[lp * NT + n]);
    cn[j * NT + m] = m == 0 ? ps : make_double2(0.0, 0.0);
    if (m == 0) {
        psi[j] = ps;
        lamn[j] = make_double2(0.0, 0.0);
        bsn[j] = ps;
    }
}

// Per-workgroup partials of the norm N0 of the initial state k_advance
// writes (c_j0 = psi_j, the other components and lambda zero).  Its
// constraint rows vanish exactly and the time couplings see zero
// coefficients, so row (j, m) holds U_0 (H psi)_j for m = 0 plus
// z_j W_m0 psi_j (the next step's field; zero without one), and
// N0 = sum_jm U_m |row_jm|^2.  One thread per point.
template <int NT>
__global__ __launch_bounds__(kThreads) void k_initial_norm(LevelGeom g, TimeOps<NT> to, int field_on,
                                                           const double2* __restrict__ psi,
                                                           const double* __restrict__ v0,
                                                           double* __restrict__ partial) {
    __shared__ double red[kThreads / 64];
    const int j = blockIdx.x * kThreads + threadIdx.x;
    double acc = 0.0;
    if (j < g.P) {
        const I3 i = point_coords(g, j);
        int nbq[6];
        nbq[0] = neighbour_of<0, -1>(g, i, j);
        nbq[1] = neighbour_of<0, 1>(g, i, j);
        nbq[2] = g.dim > 1 ? neighbour_of<1, -1>(g, i, j) : -1;
        nbq[3] = g.dim > 1 ? neighbour_of<1, 1>(g, i, j) : -1;
        nbq[4] = g.dim > 2 ? neighbour_of<2, -1>(g, i, j) : -1;
        nbq[5] = g.dim > 2 ? neighbour_of<2, 1>(g, i, j) : -1;
        const double2 own = psi[j];
        double2 nbv[6];
#pragma unroll
        for (int dir = 0; dir < 6; ++dir) nbv[dir] = psi[nbq[dir] >= 0 ? nbq[dir] : j];
        double2 lap = scl2(-2.0 * g.dim, own);
#pragma unroll
        for (int dir = 0; dir < 6; ++dir) lap = add2(lap, scl2(nbq[dir] >= 0 ? 1.0 : 0.0, nbv[dir]));
        const double2 hp = add2(scl2(-g.kin, lap), scl2(v0[j], own));
        const double zj = field_on ? zcoord(g, i) : 0.0;
#pragma unroll
        for (int m = 0; m < NT; ++m) {
            double2 r = scl2(zj * to.W[m * NT], own);
            if (m == 0) r = add2(scl2(to.U[0], hp), r);
            acc += to.U[m] * (r.x * r.x + r.y * r.y);
        }
    }
    const double tot = block_sum(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_copy_c2(const double2* __restrict__ src, double2* __restrict__ dst,
                                                      size_t n) {
    const size_t k = (size_t)blockIdx.x * kThreads + threadIdx.x;
    if (k < n) dst[k] = src[k];
}

// ---------------------------------------------------------------------------
// K10: gradients from the forward solution c and the adjoint solution mu.
//   dv0[j] += 2 Re sum_m conj(mu_jm) U_mm c_jm
//   Gpart[wg][m][n] = sum over the points the workgroup visits of z_j conj(mu_jm) c_jn
// One thread per (point slot, m) in a grid-stride loop over rounds of
// kThreads / NT points: each thread loads its own c_jm and mu_jm (every load
// coalesced), the round's rows of c and the dV0 terms meet in LDS, and the
// thread keeps row m of its points' products in registers.  The workgroup
// sums its point slots at the end, once, through LDS.
// ---------------------------------------------------------------------------
constexpr int kGradBlocks = 1536;   // workgroups of a gradient launch (at most): six per CU

template <int NT>
__global__ __launch_bounds__(kThreads, 6) void k_gradients(LevelGeom g, TimeOps<NT> to,
                                                           const double2* __restrict__ cf,
                                                           const double2* __restrict__ mu,
                                                           double* __restrict__ dv0, double2* __restrict__ Gpart) {
    constexpr int PW = kThreads / NT;  // point slots per workgroup
    __shared__ double2 cs[kThreads];   // the round's rows of c; at the end the slot sums
    __shared__ double us[kThreads];    // the round's dV0 terms U_m Re(conj(mu_jm) c_jm)
    const int t = threadIdx.x;
    const int ps = t / NT, m = t - ps * NT;
    const bool slot = ps < PW;
    const bool want_g = Gpart != nullptr;
    double um = 0.0;
#pragma unroll
    for (int n = 0; n < NT; ++n) um = n == m ? to.U[n] : um;
    double2 acc[NT];
#pragma unroll
    for (int n = 0; n < NT; ++n) acc[n] = make_double2(0.0, 0.0);
    const size_t stride = (size_t)gridDim.x * PW;
    for (size_t base = (size_t)blockIdx.x * PW; base < (size_t)g.P; base += stride) {
        const size_t j = base + ps;
        const bool on = slot && j < (size_t)g.P;
        double2 cm = make_double2(0.0, 0.0), mm = make_double2(0.0, 0.0);
        if (on) {
            cm = cf[j * NT + m];
            mm = mu[j * NT + m];
        }
        if (slot) {
            cs[t] = cm;
            us[t] = um * (mm.x * cm.x + mm.y * cm.y);
        }
        __syncthreads();
        if (on) {
            if (want_g) {
                // z conj(mu_m) c_n
                const double z = zcoord(g, point_coords(g, (int)j));
#pragma unroll
                for (int n = 0; n < NT; ++n) {
                    const double2 cn = cs[ps * NT + n];
                    acc[n].x += z * (mm.x * cn.x + mm.y * cn.y);
                    acc[n].y += z * (mm.x * cn.y - mm.y * cn.x);
                }
            }
            if (m == 0) {
                double a = 0.0;
#pragma unroll
                for (int n = 0; n < NT; ++n) a += us[ps * NT + n];
                dv0[j] += 2.0 * a;
            }
        }
        __syncthreads();
    }
    if (!want_g) return;
    // column n of the workgroup's sums: the threads m < NT add up the point slots
#pragma unroll
    for (int n = 0; n < NT; ++n) {
        if (slot) cs[t] = acc[n];
        __syncthreads();
        if (t < NT) {
            double2 sum = make_double2(0.0, 0.0);
            for (int p = 0; p < PW; ++p) sum = add2(sum, cs[p * NT + t]);
            Gpart[(size_t)blockIdx.x * NT * NT + t * NT + n] = sum;
        }
        __syncthreads();
    }
}

template <int NT>
TimeOps<NT> make_ops(const double* U, const double* W) {
    TimeOps<NT> t;
    for (int m = 0; m < NT; ++m) t.U[m] = U[m];
    for (int k = 0; k < NT * NT; ++k) t.W[k] = W ? W[k] : 0.0;
    return t;
}

inline int nblk_for(size_t n) { return (int)((n + kThreads - 1) / kThreads); }

}  // namespace

#define LAM_DISPATCH_NT(nt, CALL)    \
    switch (nt) {                     \
        case 1: { constexpr int NT = 1; CALL; } break; \
        case 2: { constexpr int NT = 2; CALL; } break; \
        case 3: { constexpr int NT = 3; CALL; } break; \
        case 4: { constexpr int NT = 4; CALL; } break; \
        case 5: { constexpr int NT = 5; CALL; } break; \
        case 6: { constexpr int NT = 6; CALL; } break; \
        case 7: { constexpr int NT = 7; CALL; } break; \
        case 8: { constexpr int NT = 8; CALL; } break; \
        default: return hipErrorInvalidValue;           \
    }

hipError_t launch_residual(int nt, const LevelGeom& g, const double* U, const double* W, int adjoint,
                           int field_on, const double2* c, const double2* lam, const double* v0, const double2* bc,
                           const double2* bg, const double2* bs, double2* rc, double2* rs, double* partial,
                           int* nparts, hipStream_t st, const int* skip, const unsigned char* bmask) {
    if (march_fits(g)) {
        const int nb = march_blocks(g);
        if (nparts) *nparts = nb;
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_residual_march<NT, false>), dim3(nb), dim3(kThreads), 0, st, g,
                                               g, make_ops<NT>(U, W), adjoint, field_on, c, lam, v0, bc, bg, bs, rc,
                                               rs, partial, skip, bmask, nullptr, nullptr, nullptr, nullptr,
                                               g.n[1] / kMarchTY, g.n[2] / kMarchTZ, march_planes(g)));
        return hipGetLastError();
    }
    const int nb = residual_blocks(nt, g.P);
    if (nparts) *nparts = nb;
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_residual<NT>, dim3(nb), dim3(kThreads), 0, st, g,
                                           make_ops<NT>(U, W), adjoint, field_on, c, lam, v0, bc, bg, bs, rc,
                                           rs, partial, skip, bmask));
    return hipGetLastError();
}

hipError_t launch_rhs_norm(int nt, int P, const double* U, const double2* rho, const double2* sig, double* partial,
                           int* nparts, hipStream_t st) {
    const int nb = residual_blocks(nt, P);
    if (nparts) *nparts = nb;
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_rhs_norm<NT>, dim3(nb), dim3(kThreads), 0, st, P,
                                           make_ops<NT>(U, nullptr), rho, sig, partial));
    return hipGetLastError();
}

hipError_t launch_block_detail(const LevelGeom& g, const double2* psi, double* out, hipStream_t st) {
    const int nblocks = g.nblk[0] * g.nblk[1] * g.nblk[2];
    if (g.bpts > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_detail, dim3(nblocks), dim3(64), 0, st, g, psi, out);
    return hipGetLastError();
}

hipError_t launch_reduce_ctl(const double* partial, int nparts, CoarseCtl* ctl, int start, double thr2,
                             int* iters_out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_ctl, dim3(1), dim3(kReduceThreads), 0, st, partial, nparts, ctl, start, thr2,
                       iters_out);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int nparts, int, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kReduceThreads), 0, st, partial, nparts, out);
    return hipGetLastError();
}

hipError_t launch_reduce_c2(const double2* partial, int nparts, int width, double2* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_c2, dim3(width), dim3(kThreads), 0, st, partial, nparts, width, out);
    return hipGetLastError();
}

hipError_t launch_residual_restrict(int nt, const LevelGeom& fine, const LevelGeom& coarse, const double* U,
                                    const double* W, int adjoint, int field_on, const double2* c,
                                    const double2* lam, const double* v0, const double2* bc, const double2* bg,
                                    const double2* bs, double2* bcc, double2* bsc, double2* zero_c,
                                    double2* zero_l, hipStream_t st) {
    if (march_fits(fine)) {
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_residual_march<NT, true>), dim3(march_blocks(fine)),
                                               dim3(kThreads), 0, st, fine, coarse, make_ops<NT>(U, W), adjoint,
                                               field_on, c, lam, v0, bc, bg, bs, nullptr, nullptr, nullptr, nullptr,
                                               nullptr, bcc, bsc, zero_c, zero_l, fine.n[1] / kMarchTY,
                                               fine.n[2] / kMarchTZ, march_planes(fine)));
        return hipGetLastError();
    }
    const int sl = 6 - fine.dim;
    const int e0 = fine.dim == 1 ? (1 << sl) : 2, e1 = fine.dim == 1 ? 1 : (fine.dim == 2 ? (1 << sl) : 2);
    const int e2 = fine.dim == 3 ? (1 << sl) : 1;
    const int t1 = (fine.n[1] + e1 - 1) / e1, t2 = (fine.n[2] + e2 - 1) / e2;
    const int nb = ((fine.n[0] + e0 - 1) / e0) * t1 * t2;
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_residual_restrict<NT>, dim3(nb), dim3(kThreads), 0, st, fine, coarse,
                                           make_ops<NT>(U, W), adjoint, field_on, c, lam, v0, bc, bg, bs, bcc, bsc,
                                           zero_c, zero_l, t1, t2, 1.0 / t1, 1.0 / t2));
    return hipGetLastError();
}

hipError_t launch_restrict(int nt, const LevelGeom& fine, const LevelGeom& coarse, const double2* rcf,
                           const double2* rsf, double2* bcc, double2* bsc, double2* zero_c, double2* zero_l,
                           hipStream_t st) {
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_restrict<NT>, dim3(nblk_for((size_t)coarse.P * (nt + 1))),
                                           dim3(kThreads), 0, st,
                                           fine, coarse, rcf, rsf, bcc, bsc, zero_c, zero_l));
    return hipGetLastError();
}

hipError_t launch_prolong(int nt, const LevelGeom& fine, const LevelGeom& coarse, int interp, const double2* cc,
                          const double2* lc, double2* cf, double2* lf, hipStream_t st) {
    // coarse tiles of 2 x 2 x 8 (8 along the last used axis)
    const int d = fine.dim;
    const int ct0 = d == 1 ? 8 : 2, ct1 = d == 1 ? 1 : (d == 2 ? 8 : 2), ct2 = d == 3 ? 8 : 1;
    const int t0 = (coarse.n[0] + ct0 - 1) / ct0, t1 = (coarse.n[1] + ct1 - 1) / ct1,
              t2 = (coarse.n[2] + ct2 - 1) / ct2;
    if (d == 3) {
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_prolong_tile<NT, 3>), dim3(t0 * t1 * t2), dim3(kThreads), 0, st,
                                               fine, coarse, interp, cc, lc, cf, lf, t1, t2));
    } else {
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_prolong_tile<NT, 0>), dim3(t0 * t1 * t2), dim3(kThreads), 0, st,
                                               fine, coarse, interp, cc, lc, cf, lf, t1, t2));
    }
    return hipGetLastError();
}

hipError_t launch_average_potential(const LevelGeom& fine, const LevelGeom& coarse, const double* vf, double* vc,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_average_potential, dim3(nblk_for(coarse.P)), dim3(kThreads), 0, st, fine, coarse, vf, vc);
    return hipGetLastError();
}

hipError_t launch_block_eig(const LevelGeom& g, const double* v0, double* V, double* e, float* Vf,
                            hipStream_t st) {
    const int nblocks = g.nblk[0] * g.nblk[1] * g.nblk[2];
    hipLaunchKernelGGL(k_block_eig, dim3(nblocks), dim3(kSweepThreads), 0, st, g, v0, V, e, Vf);
    return hipGetLastError();
}

hipError_t launch_mode_factor(int nt, const LevelGeom& g, const double* U, const double* W, const double* e,
                              const double* tf, int tf_stride, double2* Minv, float2* Minvf, hipStream_t st) {
    const int nblocks = g.nblk[0] * g.nblk[1] * g.nblk[2];
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_mode_factor<NT>, dim3(nblocks), dim3(64), 0, st, g,
                                           make_ops<NT>(U, W), e, tf, tf_stride, Minv, Minvf));
    return hipGetLastError();
}

hipError_t launch_sweep(int nt, int mixed, const SweepArgs& a, const double* U, const double* W,
                        int nblocks_colour, hipStream_t st) {
    if (nblocks_colour <= 0) return hipSuccess;
    const dim3 grid(nblocks_colour), threads(kSweepThreads);
    if (mixed && a.Minv) {
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_sweep<NT, float, true>), grid, threads, 0, st, a, make_ops<NT>(U, W)));
    } else if (mixed && (nt == 8 || nt <= 4)) {
        // two components per lane (for N_t = 5..7 its registers would spill)
        const LevelGeom& g = a.g;
        if (g.dim == 3 && g.bdim[0] == 4 && g.bdim[1] == 4 && g.bdim[2] == 4) {
            LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_sweep_pair<NT, 3>), grid, dim3(kPairThreads), 0, st, a,
                                                   make_ops<NT>(U, W)));
        } else if (g.dim == 2 && g.bdim[0] == 8 && g.bdim[1] == 8) {
            LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_sweep_pair<NT, 2>), grid, dim3(kPairThreads), 0, st, a,
                                                   make_ops<NT>(U, W)));
        } else {
            LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_sweep_pair<NT, 0>), grid, dim3(kPairThreads), 0, st, a,
                                                   make_ops<NT>(U, W)));
        }
    } else if (mixed) {
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_sweep<NT, float, false>), grid, threads, 0, st, a, make_ops<NT>(U, W)));
    } else if (a.Minv) {
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_sweep<NT, double, true>), grid, threads, 0, st, a, make_ops<NT>(U, W)));
    } else {
        LAM_DISPATCH_NT(nt, hipLaunchKernelGGL((k_sweep<NT, double, false>), grid, threads, 0, st, a, make_ops<NT>(U, W)));
    }
    return hipGetLastError();
}

hipError_t launch_init_forward(int nt, int P, const double2* psi, double2* c, double2* lam, double2* bs,
                               hipStream_t st) {
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_init_forward<NT>, dim3(nblk_for((size_t)P * nt)), dim3(kThreads), 0,
                                           st, P, psi, c, lam, bs));
    return hipGetLastError();
}

hipError_t launch_init_zero(int nt, int P, double2* c, double2* lam, hipStream_t st) {
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_init_zero<NT>, dim3(nblk_for((size_t)P * nt)), dim3(kThreads), 0, st, P,
                                           c, lam));
    return hipGetLastError();
}

hipError_t launch_end_eval(int nt, int P, const double2* c, double2* psi, hipStream_t st) {
    LAM_DISPATCH_NT(nt,
                    hipLaunchKernelGGL(k_end_eval<NT>, dim3(nblk_for(P)), dim3(kThreads), 0, st, P, c, psi));
    return hipGetLastError();
}

hipError_t launch_advance(int nt, const LevelGeom& g, const double* U, const double* W, const double2* c,
                          const double* v0, double2* psi, double2* cn, double2* lamn, double2* bsn,
                          double* partial, int* nparts, hipStream_t st) {
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_advance<NT>, dim3(residual_blocks(nt, g.P)), dim3(kThreads), 0, st,
                                           g.P, c, psi, cn, lamn, bsn));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // at most residual_blocks(nt, P) partials, the capacity of a residual launch's
    const int nb = nblk_for(g.P);
    if (nparts) *nparts = nb;
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_initial_norm<NT>, dim3(nb), dim3(kThreads), 0, st, g,
                                           make_ops<NT>(U, W), W ? 1 : 0, psi, v0, partial));
    return hipGetLastError();
}

hipError_t launch_copy_c2(const double2* src, double2* dst, size_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_c2, dim3(nblk_for(n)), dim3(kThreads), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_gradients(int nt, const LevelGeom& g, const double* U, const double2* cfwd, const double2* mu,
                            double* dv0, double2* Gpart, int* nparts, hipStream_t st) {
    // at most one workgroup per kThreads points: the partial buffer holds that many
    const int nb = std::min(nblk_for(g.P), kGradBlocks);
    if (nparts) *nparts = nb;
    LAM_DISPATCH_NT(nt, hipLaunchKernelGGL(k_gradients<NT>, dim3(nb), dim3(kThreads), 0, st, g,
                                           make_ops<NT>(U, nullptr), cfwd, mu, dv0, Gpart));
    return hipGetLastError();
}

}  // namespace lam
