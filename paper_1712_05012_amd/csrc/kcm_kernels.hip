// kcm_kernels.hip -- gfx950 kernels of one KCM iteration.
//
//   k_tau       one thread per joint: joint torques of the pending forces,
//               tau_k = u_k . (T_k - p_k x F_k) (eqs KCM_01-KCM_06), with the
//               wrench of later atom workgroups from a suffix (row) scan
//               (eq 04_9).
//   k_stepfk    one thread per joint: the compliance step (eq KCM_07), then
//               forward kinematics of the new angles as an ordered prefix
//               scan of rigid transforms inside each joint block (eqs
//               kin_02-kin_04, r1; prefix computation item 1 of Sec. 3.5).
//   k_place     one thread per atom: link transforms (products of the
//               earlier joint blocks composed in front of the block-local
//               ones), r_a = G_link(a) r0_a, per-workgroup bounding box of
//               the new positions.
//   k_cellkey   one thread per atom: the cell grid of Sec. 3.2 sized from
//               that bounding box (in every workgroup of a small chain, in
//               k_grid before it for a large one), cell key, count and the
//               atom's place among its cell's arrivals.
//   k_cellscan  one workgroup per 4096 cells: exclusive scan of the counts
//               inside the chunk, and its total.
//   (k_scatter and k_rank add the chunk offsets; k_rank writes the starts.)
//   k_scatter   one thread per atom: counting-sort scatter by cell key.
//   k_rank      one thread per atom: stable slot inside the cell, gather.
//   k_force     one wave per atom, atoms in cell order: stencil candidates
//               in FP64, Coulomb + LJ (eqs 02-03_9), solvation neighbours in
//               LDS, and the SASA enumeration of Algorithm 1 with the C-state
//               rules (Sec. 3.4): coverage counts with four samples per lane,
//               the displaced tests of critical samples inline and those of
//               exposed samples with one lane per neighbour.  Solvation
//               events are scattered as fixed-point integers.
//   k_wrench    one thread per atom: wrench (F, r x F), the suffix sum inside
//               the workgroup and the workgroup-local part of each torque.
#include "kcm_internal.h"

#include <float.h>
#include <math.h>

namespace kcm {

constexpr int WAVE = 64;
constexpr double PI_D = 3.14159265358979323846;
// Half width of the FP32 decision band of the mixed form: a sample test whose
// FP32 value lies this close to its threshold is decided again in FP64.  The
// FP32 error of the tested quantity stays below ~5e-6 A for offsets < 16 A.
constexpr float MIXED_BAND = 4.0e-5f;

// ---------------------------------------------------------------------------
// rigid transforms (rotation R row-major, translation t): x -> R x + t
// ---------------------------------------------------------------------------
struct Xf {
    double r[9];
    double t[3];
};

__device__ __forceinline__ Xf xf_identity()
{
    Xf x;
#pragma unroll
    for (int k = 0; k < 9; ++k) x.r[k] = (k % 4 == 0) ? 1.0 : 0.0;
    x.t[0] = x.t[1] = x.t[2] = 0.0;
    return x;
}

// (A o B)(x) = A(B(x))
__device__ __forceinline__ Xf xf_mul(const Xf &A, const Xf &B)
{
    Xf C;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
            C.r[3 * i + j] = A.r[3 * i] * B.r[j] + A.r[3 * i + 1] * B.r[3 + j] + A.r[3 * i + 2] * B.r[6 + j];
        C.t[i] = A.r[3 * i] * B.t[0] + A.r[3 * i + 1] * B.t[1] + A.r[3 * i + 2] * B.t[2] + A.t[i];
    }
    return C;
}

__device__ __forceinline__ Xf xf_shfl_up(const Xf &x, int d)
{
    Xf y;
#pragma unroll
    for (int k = 0; k < 9; ++k) y.r[k] = __shfl_up(x.r[k], d, WAVE);
#pragma unroll
    for (int k = 0; k < 3; ++k) y.t[k] = __shfl_up(x.t[k], d, WAVE);
    return y;
}

__device__ __forceinline__ void xf_store(double *p, const Xf &x)
{
#pragma unroll
    for (int k = 0; k < 9; ++k) p[k] = x.r[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) p[9 + k] = x.t[k];
}

__device__ __forceinline__ Xf xf_load(const double *p)
{
    Xf x;
#pragma unroll
    for (int k = 0; k < 9; ++k) x.r[k] = p[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) x.t[k] = p[9 + k];
    return x;
}

__device__ __forceinline__ int link_of_atom(int a)
{
    const int res = a / APR, slot = a - res * APR;
    return 2 * res + (slot < 2 ? 0 : (slot < 8 ? 1 : 2));
}

// ---------------------------------------------------------------------------
// block-wide helpers (blockDim.x a multiple of 64, at most 1024)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}
__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmax(v, __shfl_xor(v, d, WAVE));
    return v;
}
__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v = fmin(v, __shfl_xor(v, d, WAVE));
    return v;
}
__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// Sum of K doubles over the block; the result is returned to every thread.
// Fixed reduction order, so it is deterministic.  scratch: [16][K].
template <int K>
__device__ void block_sum(double (&v)[K], double *scratch)
{
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < K; ++k) scratch[w * K + k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += scratch[i * K + k];
        v[k] = s;
    }
    __syncthreads();
}

__device__ double block_max(double v, double *scratch)
{
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    v = wave_max(v);
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    double m = -DBL_MAX;
    for (int i = 0; i < nw; ++i) m = fmax(m, scratch[i]);
    __syncthreads();
    return m;
}

// Exclusive prefix sum of one int per thread over the block; *total gets the sum.
__device__ int block_excl_scan(int v, int *scratch, int *total)
{
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    int x = v;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    __syncthreads();
    if (lane == WAVE - 1) scratch[w] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) base += scratch[i];
        tot += scratch[i];
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}


__device__ __forceinline__ int find_block_owner(const int32_t *off, int n, int b)
{
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// The kernels after the step run a chain iff the step kept it running and its
// grid for this iteration could be sized.
__device__ __forceinline__ bool running(const ChainStats *st) { return st->run && !st->grid_bad; }

__device__ __forceinline__ int cell_of(const Grid &g, const double4 &r)
{
    int cx = (int)floor((r.x - g.origin[0]) * g.inv_cell);
    int cy = (int)floor((r.y - g.origin[1]) * g.inv_cell);
    int cz = (int)floor((r.z - g.origin[2]) * g.inv_cell);
    cx = min(max(cx, 0), g.dims[0] - 1);
    cy = min(max(cy, 0), g.dims[1] - 1);
    cz = min(max(cz, 0), g.dims[2] - 1);
    return (cz * g.dims[1] + cy) * g.dims[0] + cx;
}

constexpr double GRID_MARGIN = 2.0;  // A added around the bounding box of the placed atoms
constexpr int LINKS_PER_BLOCK = 56;  // links touched by ATOM_BLOCK consecutive atoms (at most 53)

// First atom moved by joint j: the first atom of link j+1 (C-alpha for phi,
// C for psi).
__device__ __forceinline__ int first_atom_of_joint(int j) { return APR * (j >> 1) + ((j & 1) ? 8 : 2); }
__device__ __forceinline__ int first_atom_of_link(int l) { return l == 0 ? 0 : first_atom_of_joint(l - 1); }

__device__ __forceinline__ Xf xf_shfl_idx(const Xf &x, int src)
{
    Xf y;
#pragma unroll
    for (int k = 0; k < 9; ++k) y.r[k] = __shfl(x.r[k], src, WAVE);
#pragma unroll
    for (int k = 0; k < 3; ++k) y.t[k] = __shfl(x.t[k], src, WAVE);
    return y;
}

// Writes the link transform G_{j+1} and the current axis (u_j, p_j) of joint j.
__device__ __forceinline__ void fk_emit(const Xf &G, int j, const double4 *__restrict__ joint0, double *__restrict__ xform,
                                        double4 *__restrict__ jcur)
{
    xf_store(xform + 12 * (j + 1), G);
    const double4 u0 = joint0[2 * j], p0 = joint0[2 * j + 1];
    double4 u, p;
    u.x = G.r[0] * u0.x + G.r[1] * u0.y + G.r[2] * u0.z;
    u.y = G.r[3] * u0.x + G.r[4] * u0.y + G.r[5] * u0.z;
    u.z = G.r[6] * u0.x + G.r[7] * u0.y + G.r[8] * u0.z;
    u.w = 0.0;
    p.x = G.r[0] * p0.x + G.r[1] * p0.y + G.r[2] * p0.z + G.t[0];
    p.y = G.r[3] * p0.x + G.r[4] * p0.y + G.r[5] * p0.z + G.t[1];
    p.z = G.r[6] * p0.x + G.r[7] * p0.y + G.r[8] * p0.z + G.t[2];
    p.w = 0.0;
    jcur[2 * j] = u;
    jcur[2 * j + 1] = p;
}

// Rodrigues rotation about unit u by angle (th - pi) and the translation that
// keeps the axis point p fixed.
__device__ __forceinline__ Xf joint_xf_of(const double4 &u, const double4 &p, double th)
{
    double s, c;
    sincos(th - PI_D, &s, &c);
    const double k = 1.0 - c;
    Xf x;
    x.r[0] = c + u.x * u.x * k;       x.r[1] = u.x * u.y * k - u.z * s; x.r[2] = u.x * u.z * k + u.y * s;
    x.r[3] = u.y * u.x * k + u.z * s; x.r[4] = c + u.y * u.y * k;       x.r[5] = u.y * u.z * k - u.x * s;
    x.r[6] = u.z * u.x * k - u.y * s; x.r[7] = u.z * u.y * k + u.x * s; x.r[8] = c + u.z * u.z * k;
#pragma unroll
    for (int i = 0; i < 3; ++i) x.t[i] = ((&p.x)[i]) - (x.r[3 * i] * p.x + x.r[3 * i + 1] * p.y + x.r[3 * i + 2] * p.z);
    return x;
}

// Grid of Sec. 3.2 from the per-workgroup bounding boxes of the placed atoms,
// plus a margin; the cell edge starts at max(cell_min, reach / MAX_REACH) and
// grows until the grid fits the chain's cell capacity.  Block-wide (any block
// size); returns false (and a one-cell grid) when the box is not finite or
// cannot be covered.  s_red: [nw * 6].
// The grid for the bounding box [lo, hi] of the placed atoms, plus a margin
// (one thread); *ok stays true iff it could be sized within the capacity.
__device__ Grid size_grid(const ChainDev *cd, const double lo[3], const double hi[3], bool *ok)
{
    double L3[3], H3[3];
    for (int k = 0; k < 3; ++k) {
        L3[k] = lo[k] - GRID_MARGIN;
        H3[k] = hi[k] + GRID_MARGIN;
        *ok = *ok && isfinite(L3[k]) && isfinite(H3[k]) && H3[k] >= L3[k] && (H3[k] - L3[k]) < 1e7;
    }
    const double reach_len = fmax(cd->cutoff, 2.0 * cd->roff_max + cd->delta_r) + 1e-7;
    double cell = fmax(cd->cell_min, reach_len / MAX_REACH);
    long long dims[3] = {1, 1, 1};
    for (int it = 0; *ok && it < 200; ++it) {
        for (int k = 0; k < 3; ++k) dims[k] = (long long)floor((H3[k] - L3[k]) / cell) + 1;
        if (dims[0] * dims[1] * dims[2] <= cd->cap_cells) break;
        cell *= 1.2599210498948732;
    }
    *ok = *ok && dims[0] * dims[1] * dims[2] <= cd->cap_cells;
    Grid g;
    for (int k = 0; k < 3; ++k) { g.origin[k] = *ok ? L3[k] : 0.0; g.dims[k] = *ok ? (int)dims[k] : 1; }
    g.cell = cell;
    g.inv_cell = 1.0 / cell;
    g.reach = max(1, (int)ceil(reach_len / cell - 1e-9));
    g.reach_len = reach_len;
    g.n_cells = *ok ? (int)(dims[0] * dims[1] * dims[2]) : 1;
    g.pad = 0;
    return g;
}

__device__ bool grid_from_parts(const ChainDev *cd, Grid *out, double *s_red, int *s_ok)
{
    const int n = cd->n_atoms;
    const int nblk = (n + ATOM_BLOCK - 1) / ATOM_BLOCK;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (WAVE - 1), w = tid / WAVE, nw = nt / WAVE;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    bool fin = true;
    for (int b = tid; b < nblk; b += nt)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double l = cd->bbox_part[6 * b + k], h = cd->bbox_part[6 * b + 3 + k];
            fin = fin && isfinite(l) && isfinite(h);
            lo[k] = fmin(lo[k], l);
            hi[k] = fmax(hi[k], h);
        }
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
    const bool bad_w = __any(!fin);
    if (tid == 0) *s_ok = 1;
    __syncthreads();
    if (lane == 0) {
        for (int k = 0; k < 3; ++k) { s_red[w * 6 + k] = lo[k]; s_red[w * 6 + 3 + k] = hi[k]; }
        if (bad_w) *s_ok = 0;
    }
    __syncthreads();
    if (w == 0) {
        // wave 0 reduces the wave partials, lane i holding wave i's
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = wave_min(lane < nw ? s_red[lane * 6 + k] : DBL_MAX);
            hi[k] = wave_max(lane < nw ? s_red[lane * 6 + 3 + k] : -DBL_MAX);
        }
    }
    if (tid == 0) {
        bool ok = *s_ok != 0;
        *out = size_grid(cd, lo, hi, &ok);
        *s_ok = ok ? 1 : 0;
    }
    __syncthreads();
    return *s_ok != 0;
}

// ---------------------------------------------------------------------------
// k_tau: joint torques of the pending forces, one thread per joint
// ---------------------------------------------------------------------------
// k_wrench left in tau[j] the part of tau_j from the atoms of the workgroup
// that holds j's first downstream atom, and in wrench_part[b] the wrench sum
// (F, r x F) of atom workgroup b.  The rest comes from every later workgroup
// (the row scan of eq 04_9): tau_j += u_j . (T_later - p_j x F_later), eqs
// KCM_01-KCM_06.
__global__ __launch_bounds__(JOINT_BLOCK) void k_tau(Batch bt)
{
    const int c = find_block_owner(bt.jblk_off, bt.n_chains, blockIdx.x);
    const ChainDev *cd = bt.table[c];
    ChainStats *st = cd->stats;
    if (!st->active || !st->pending_post) return;
    __shared__ double s_red[(JOINT_BLOCK / WAVE) * 6];
    __shared__ double s_S[8][6];
    const int jb = blockIdx.x - bt.jblk_off[c];
    const int tid = threadIdx.x;
    if (jb >= cd->n_bb_blocks) {
        // a block of side-chain joints: k_wrench left each chi torque whole
        const int jc = (jb - cd->n_bb_blocks) * JOINT_BLOCK + tid, j = cd->n_joints + jc;
        double tabs = 0.0, bad = 0.0;
        if (jc < cd->n_chi) {
            const double t = cd->tau[j];
            if (!isfinite(t)) bad = 1.0;
            if (cd->mask[j]) tabs = fabs(t);
        }
        const double tmax = block_max(tabs, s_red);
        const double anybad = block_max(bad, s_red);
        if (tid == 0) {
            cd->tmax_part[jb] = tmax;
            cd->bad_part[jb] = anybad > 0.0 ? 1 : 0;
        }
        return;
    }
    const int J = cd->n_joints, n = cd->n_atoms;
    const int nblk = (n + ATOM_BLOCK - 1) / ATOM_BLOCK;
    const double *__restrict__ part = cd->wrench_part;
    // the joints of this workgroup take their later-workgroup wrench after
    // atom workgroups blo..bhi (at most 6 of them)
    const int jlo = jb * JOINT_BLOCK, jhi = min(J, jlo + JOINT_BLOCK) - 1;
    const int blo = first_atom_of_joint(jlo) / ATOM_BLOCK, bhi = first_atom_of_joint(jhi) / ATOM_BLOCK;
    __shared__ double s_P[8][6];
    if (tid < 6 * (bhi - blo + 1)) s_P[tid / 6][tid % 6] = part[WPART * (blo + tid / 6) + tid % 6];
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int b = bhi + 1 + tid; b < nblk; b += JOINT_BLOCK)
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] += part[WPART * b + k];
    block_sum<6>(v, s_red);
    if (tid < 6) {
        // suffix over the touched workgroups, one wrench component per thread
        double x = v[tid];
        for (int b = bhi; b >= blo; --b) {
            s_S[b - blo][tid] = x;
            x += s_P[b - blo][tid];
        }
    }
    __syncthreads();

    const int j = jlo + tid;
    double tabs = 0.0, bad = 0.0;
    if (j < J) {
        const double *S = s_S[first_atom_of_joint(j) / ATOM_BLOCK - blo];
        const double4 u = cd->jcur[2 * j], p = cd->jcur[2 * j + 1];
        const double mx = S[3] - (p.y * S[2] - p.z * S[1]);
        const double my = S[4] - (p.z * S[0] - p.x * S[2]);
        const double mz = S[5] - (p.x * S[1] - p.y * S[0]);
        const double t = cd->tau[j] + (u.x * mx + u.y * my + u.z * mz);
        cd->tau[j] = t;
        if (!isfinite(t)) bad = 1.0;
        if (cd->mask[j]) tabs = fabs(t);
    }
    const double tmax = block_max(tabs, s_red);
    const double anybad = block_max(bad, s_red);
    if (tid == 0) {
        cd->tmax_part[jb] = tmax;
        cd->bad_part[jb] = anybad > 0.0 ? 1 : 0;
    }
    if (jb == 0) {
        // energies and the non-finite force flag of the pending forces
        double E[4] = {0, 0, 0, 0};
        for (int b = tid; b < nblk; b += JOINT_BLOCK)
#pragma unroll
            for (int k = 0; k < 4; ++k) E[k] += part[WPART * b + 6 + k];
        block_sum<4>(E, s_red);
        if (tid == 0) {
            st->e_elec = E[0];
            st->e_vdw = E[1];
            st->e_cav = E[2];
            st->post_bad = E[3] > 0.0 ? 1 : 0;
        }
    }
}

// ---------------------------------------------------------------------------
// k_stepfk: compliance step of the pending forces (eq KCM_07), then the
// kinematics of the new angles inside each joint block (eqs kin_02-kin_04,
// r1): xform_loc[j] = T_{jlo} o ... o T_j by an ordered scan, and the block
// product in blk_xf.  k_place composes the products of earlier blocks in
// front (prefix computation, item 1 of Sec. 3.5).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(JOINT_BLOCK) void k_stepfk(Batch bt, int mode)
{
    const int c = find_block_owner(bt.jblk_off, bt.n_chains, blockIdx.x);
    const ChainDev *cd = bt.table[c];
    ChainStats *st = cd->stats;
    if (!st->active) return;
    if (mode == MODE_BOOT && !st->need_grid) return;
    __shared__ double s_red[JOINT_BLOCK / WAVE];
    __shared__ double s_x[JOINT_BLOCK / WAVE][12];
    const int jb = blockIdx.x - bt.jblk_off[c];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int J = cd->n_joints;
    // backbone blocks first; the blocks after them hold the side-chain joints,
    // which step with the others but are not part of the chain's scan
    const bool chi_block = jb >= cd->n_bb_blocks;
    if (chi_block && mode == MODE_BOOT) return;
    const int j = chi_block ? J + (jb - cd->n_bb_blocks) * JOINT_BLOCK + tid : jb * JOINT_BLOCK + tid;
    const bool valid = chi_block ? j < J + cd->n_chi : j < J;
    double th = valid ? cd->theta[j] : 0.0;
    const bool lead = jb == 0 && tid == 0;

    if (mode != MODE_BOOT && st->pending_post) {
        const int nb = cd->n_bb_blocks + (cd->n_chi + JOINT_BLOCK - 1) / JOINT_BLOCK;
        double tm = 0.0, bad = 0.0;
        for (int b = tid; b < nb; b += JOINT_BLOCK) {
            tm = fmax(tm, cd->tmax_part[b]);
            if (cd->bad_part[b]) bad = 1.0;
        }
        tm = block_max(tm, s_red);
        bad = block_max(bad, s_red);
        if (bad > 0.0 || st->post_bad) {
            if (lead) {
                st->status = -4;
                st->run = 0;
            }
            return;
        }
        const double kappa = cd->kappa, smax = cd->max_step;
        double scale;
        if (cd->step_rule == 1) scale = tm > 0.0 ? smax / tm : 0.0;
        else if (cd->step_rule == 2) scale = kappa;
        else scale = (kappa * tm > smax) ? smax / tm : kappa;
        if (valid) {
            const double d = cd->mask[j] ? scale * cd->tau[j] : 0.0;
            cd->dtheta[j] = d;
            double t = th + d;
            if (t > PI_D) t -= 2.0 * PI_D;
            if (t <= -PI_D) t += 2.0 * PI_D;
            th = t;
            cd->theta[j] = t;
        }
        if (lead) {
            // max |dtheta| over the moving joints is scale * max |tau| exactly
            const double mxd = scale * tm;
            st->max_tau = tm;
            st->max_dtheta = mxd;
            st->iterations += 1;
            if (st->nbr_overflow) st->status = -6;
            int go = 1;
            if (st->tol > 0.0 && mxd < st->tol) {
                st->converged = 1;
                go = 0;
            }
            if (st->iterations >= st->iter_limit) go = 0;
            st->run = go;
        }
    } else if (lead && mode != MODE_BOOT) {
        st->run = 1;
    }
    if (mode == MODE_FINAL || chi_block) return;

    Xf x = xf_identity();
    if (valid) x = joint_xf_of(cd->joint0[2 * j], cd->joint0[2 * j + 1], th);
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        Xf y = xf_shfl_up(x, d);
        if (lane >= d) x = xf_mul(y, x);
    }
    if (lane == WAVE - 1) xf_store(s_x[w], x);
    __syncthreads();
    if (w > 0) {
        Xf pre = xf_load(s_x[0]);
        for (int i = 1; i < w; ++i) pre = xf_mul(pre, xf_load(s_x[i]));
        x = xf_mul(pre, x);
    }
    if (valid) xf_store(cd->xform_loc + 12 * j, x);
    if (tid == min(J - jb * JOINT_BLOCK, JOINT_BLOCK) - 1) xf_store(cd->blk_xf + 12 * jb, x);
}

// ---------------------------------------------------------------------------
// k_place: link transforms of this workgroup's links, positions
// r_a = G_link(a) r0_a, cell keys and counts, bounding box
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(ATOM_BLOCK) void k_place(Batch bt, int mode)
{
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    ChainStats *st = cd->stats;
    const int lb = blockIdx.x - bt.blk_off[c];
    // the step and torque kernels of this iteration have consumed the pending forces
    if (mode == MODE_ITER && lb == 0 && threadIdx.x == 0) st->pending_post = 0;
    if (mode == MODE_BOOT ? !(st->active && st->need_grid) : !running(st)) return;
    __shared__ double s_G[LINKS_PER_BLOCK][12];
    __shared__ double s_c[2][12];
    __shared__ double s_bb[ATOM_BLOCK / WAVE][6];
    __shared__ int s_bad[ATOM_BLOCK / WAVE];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int n = cd->n_atoms;
    const int a0 = lb * ATOM_BLOCK, a1 = min(n, a0 + ATOM_BLOCK) - 1;
    const int l_lo = link_of_atom(a0), l_hi = link_of_atom(a1);
    // link l (>= 1) needs the product of the joint blocks before joint l-1
    const int jb_lo = (max(l_lo, 1) - 1) / JOINT_BLOCK, jb_hi = (max(l_hi, 1) - 1) / JOINT_BLOCK;
    if (w == 0) {
        Xf acc = xf_identity();
        for (int base = 0; base < jb_hi; base += WAVE) {
            Xf x = (base + lane < jb_hi) ? xf_load(cd->blk_xf + 12 * (base + lane)) : xf_identity();
#pragma unroll
            for (int d = 1; d < WAVE; d <<= 1) {
                Xf y = xf_shfl_up(x, d);
                if (lane >= d) x = xf_mul(y, x);
            }
            if (base > 0) x = xf_mul(acc, x);
            if (base + lane == jb_lo - 1) xf_store(s_c[0], x);
            if (base + lane == jb_hi - 1) xf_store(s_c[1], x);
            acc = xf_shfl_idx(x, WAVE - 1);
        }
        if (lane == 0) {
            if (jb_lo == 0) xf_store(s_c[0], xf_identity());
            if (jb_hi == 0) xf_store(s_c[1], xf_identity());
        }
    }
    __syncthreads();
    const int nL = l_hi - l_lo + 1;
    for (int t = tid; t < nL; t += ATOM_BLOCK) {
        const int l = l_lo + t;
        Xf G = xf_identity();
        if (l > 0) {
            const int j = l - 1;
            G = xf_mul(xf_load(s_c[j / JOINT_BLOCK == jb_lo ? 0 : 1]), xf_load(cd->xform_loc + 12 * j));
        }
        xf_store(s_G[t], G);
        const int fa = first_atom_of_link(l);
        if (fa >= a0 && fa <= a1) {
            if (l == 0) xf_store(cd->xform, G);
            else fk_emit(G, l - 1, cd->joint0, cd->xform, cd->jcur);
        }
    }
    __syncthreads();

    const int a = a0 + tid;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    bool fin = true;
    if (a <= a1) {
        const double *L = s_G[link_of_atom(a) - l_lo];
        double4 q = cd->r0[a];
        const int res = a / APR, slot = a - res * APR;
        if (cd->n_chi && slot >= 5 && slot <= 7) {
            // side-chain joint chi of the residue (dihedral N-CA-CB-HB1, 60
            // degrees in the zero position): HB1..HB3 turn about CA->CB, here
            // in the zero-position frame before the link transform
            const double4 ca = cd->r0[res * APR + 2], cb = cd->r0[res * APR + 4];
            double ux = cb.x - ca.x, uy = cb.y - ca.y, uz = cb.z - ca.z;
            const double inv = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
            ux *= inv; uy *= inv; uz *= inv;
            double sn, cs;
            sincos(cd->theta[cd->n_joints + res] - PI_D / 3.0, &sn, &cs);
            const double vx = q.x - cb.x, vy = q.y - cb.y, vz = q.z - cb.z;
            const double dot = ux * vx + uy * vy + uz * vz;
            const double wx = uy * vz - uz * vy, wy = uz * vx - ux * vz, wz = ux * vy - uy * vx;
            q.x = cb.x + vx * cs + wx * sn + ux * dot * (1.0 - cs);
            q.y = cb.y + vy * cs + wy * sn + uy * dot * (1.0 - cs);
            q.z = cb.z + vz * cs + wz * sn + uz * dot * (1.0 - cs);
        }
        double4 r;
        r.x = L[0] * q.x + L[1] * q.y + L[2] * q.z + L[9];
        r.y = L[3] * q.x + L[4] * q.y + L[5] * q.z + L[10];
        r.z = L[6] * q.x + L[7] * q.y + L[8] * q.z + L[11];
        r.w = 0.0;
        cd->r[a] = r;
        fin = isfinite(r.x) && isfinite(r.y) && isfinite(r.z);
        if (mode == MODE_ITER) {
            cd->f_cav[3 * a] = 0;
            cd->f_cav[3 * a + 1] = 0;
            cd->f_cav[3 * a + 2] = 0;
        }
        lo[0] = r.x; lo[1] = r.y; lo[2] = r.z;
        hi[0] = r.x; hi[1] = r.y; hi[2] = r.z;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
    const bool bad_w = __any(!fin);
    if (lane == 0) {
        for (int k = 0; k < 3; ++k) { s_bb[w][k] = lo[k]; s_bb[w][3 + k] = hi[k]; }
        s_bad[w] = bad_w ? 1 : 0;
    }
    __syncthreads();
    if (tid < 6) {
        const int k = tid;
        double v = s_bb[0][k];
        int bad = s_bad[0];
        for (int i = 1; i < ATOM_BLOCK / WAVE; ++i) {
            v = (k < 3) ? fmin(v, s_bb[i][k]) : fmax(v, s_bb[i][k]);
            bad |= s_bad[i];
        }
        cd->bbox_part[6 * lb + k] = bad ? NAN : v;
    }
}

// ---------------------------------------------------------------------------
// k_grid and k_cellkey: this iteration's grid of Sec. 3.2, sized from the
// bounding box of the positions just placed plus a margin, then every atom's
// cell key and the cell counts.  The grid is a function of the current
// conformation alone, so a chain rebuilt from saved angles continues exactly
// as the original.  Two launch forms with the same grid and keys: for large
// batches one wave per chain sizes the grid (k_grid) and the key workgroups
// read it; for small ones, where a launch costs more than the redundant work,
// wave 0 of every key workgroup sizes it and the first one stores it.
// ---------------------------------------------------------------------------
// the grid from the chain's bounding-box partials (one wave; lane 0 gets it)
__device__ __forceinline__ Grid wave_grid(const ChainDev *cd, bool *ok)
{
    const int lane = (int)threadIdx.x & (WAVE - 1), nblk = (cd->n_atoms + ATOM_BLOCK - 1) / ATOM_BLOCK;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    bool fin = true;
    for (int b = lane; b < nblk; b += WAVE)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double l = cd->bbox_part[6 * b + k], h = cd->bbox_part[6 * b + 3 + k];
            fin = fin && isfinite(l) && isfinite(h);
            lo[k] = fmin(lo[k], l);
            hi[k] = fmax(hi[k], h);
        }
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
    *ok = !__any(!fin);
    Grid g{};
    if (lane == 0) g = size_grid(cd, lo, hi, ok);
    return g;
}

__device__ __forceinline__ void store_grid(ChainDev *cd, ChainStats *st, const Grid &g, bool ok)
{
    if (ok) {
        *cd->grid = g;
    } else {
        st->status = -4;
        st->grid_bad = 1;
    }
}

__global__ __launch_bounds__(WAVE) void k_grid(Batch bt)
{
    ChainDev *cd = bt.table[blockIdx.x];
    ChainStats *st = cd->stats;
    if (!running(st)) return;
    bool ok;
    const Grid g = wave_grid(cd, &ok);
    if (threadIdx.x == 0) store_grid(cd, st, g, ok);
}

template <bool OWN_GRID>
__global__ __launch_bounds__(ATOM_BLOCK) void k_cellkey(Batch bt)
{
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    ChainStats *st = cd->stats;
    // with OWN_GRID, grid_bad is set by this kernel: a workgroup that sees it
    // set by the first one would have found the same failure itself
    if (!running(st)) return;
    __shared__ int s_ok;
    __shared__ Grid s_g;
    const int lb = blockIdx.x - bt.blk_off[c];
    if (OWN_GRID) {
        if (threadIdx.x < WAVE) {
            bool ok;
            const Grid g = wave_grid(cd, &ok);
            if (threadIdx.x == 0) {
                s_g = g;
                s_ok = ok ? 1 : 0;
                if (lb == 0) store_grid(cd, st, g, ok);
            }
        }
        __syncthreads();
        if (!s_ok) return;
    } else if (threadIdx.x == 0) {
        s_g = *cd->grid;
    }
    // Atoms of the workgroup that share a cell take one count atomic between
    // them: an LDS table (open addressing on the key, twice as many slots as
    // atoms, so a probe always ends) gives each atom its rank among them, the
    // first adds their number to the cell's count, and each atom's place among
    // the cell's arrivals is the returned base plus its rank.
    constexpr int HSLOTS = 2 * ATOM_BLOCK;
    __shared__ int s_hkey[HSLOTS], s_hcnt[HSLOTS], s_hbase[HSLOTS];
    for (int h = threadIdx.x; h < HSLOTS; h += ATOM_BLOCK) {
        s_hkey[h] = -1;
        s_hcnt[h] = 0;
    }
    __syncthreads();
    const int a = lb * ATOM_BLOCK + threadIdx.x;
    const bool valid = a < cd->n_atoms;
    int key = 0, slot = 0, rank = 0;
    if (valid) {
        key = cell_of(s_g, cd->r[a]);
        cd->cell_key[a] = key;
        slot = (int)(((unsigned)key * 2654435761u) >> 23) & (HSLOTS - 1);
        for (;;) {
            const int prev = atomicCAS(&s_hkey[slot], -1, key);
            if (prev == -1 || prev == key) break;
            slot = (slot + 1) & (HSLOTS - 1);
        }
        rank = atomicAdd(&s_hcnt[slot], 1);
    }
    __syncthreads();
    if (valid && rank == 0) s_hbase[slot] = atomicAdd(&cd->cell_count[key], s_hcnt[slot]);
    __syncthreads();
    // kept for the scatter in the sorted-index array (free until the rank
    // kernel fills it)
    if (valid) cd->s_idx[a] = s_hbase[slot] + rank;
}

// ---------------------------------------------------------------------------
// k_gridboot: first grid of a chain whose conformation has no grid yet
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(CHAIN_THREADS) void k_gridboot(Batch bt)
{
    ChainDev *cd = bt.table[blockIdx.x];
    ChainStats *st = cd->stats;
    if (!st->active || !st->need_grid) return;
    __shared__ double s_red[CHAIN_THREADS / WAVE * 6];
    __shared__ int s_ok;
    const bool ok = grid_from_parts(cd, cd->grid, s_red, &s_ok);
    if (threadIdx.x == 0) {
        st->need_grid = 0;
        if (!ok) {
            st->status = -4;
            st->active = 0;
            st->run = 0;
        }
    }
}

// k_finish: the call's last post phase is applied; the chain's state for the
// next call is its run flag.
__global__ void k_finish(Batch bt)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bt.n_chains) return;
    ChainStats *st = bt.table[c]->stats;
    st->pending_post = 0;
    st->active = running(st);
}

// k_stats_gather: the records of every chain of the batch into one array, so
// that the host reads them back with a single copy.
__global__ void k_stats_gather(Batch bt, ChainStats *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bt.n_chains) return;
    out[c] = *bt.table[c]->stats;
}

// k_fold_control: FOLD_BEGIN keeps the chain's own stopping rule
// (kcm_set_limits) aside and arms every chain for a fold of at most max_iter
// iterations that stops below tol (a chain with a failure status stays
// stopped); FOLD_END puts the chain's own rule back and leaves every chain
// steppable again unless it converged, failed or reached its own limit.
__global__ void k_fold_control(Batch bt, int mode, double tol, int64_t max_iter)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bt.n_chains) return;
    ChainStats *st = bt.table[c]->stats;
    if (mode == FOLD_BEGIN) {
        const int go = st->status == 0 && max_iter > 0 ? 1 : 0;
        st->saved_tol = st->tol;
        st->saved_limit = st->iter_limit;
        st->tol = tol;
        st->iter_limit = st->iterations + max_iter;
        st->converged = 0;
        st->active = go;
        st->run = go;
    } else {
        st->tol = st->saved_tol;
        st->iter_limit = st->saved_limit;
        const int again = st->status == 0 && !st->converged && st->iterations < st->iter_limit ? 1 : 0;
        st->active = again;
        st->run = again;
    }
}

// ---------------------------------------------------------------------------
// Monte Carlo minimization over the descent (the hybrid of Monte Carlo
// sampling and steepest descent among the search improvements of Sec. 4, in
// the form of Li and Scheraga): perturb the accepted angles, descend, keep the
// descended state by the Metropolis rule on its energy.  Three small kernels
// around the ordinary iterations; the random numbers are inputs.
// ---------------------------------------------------------------------------
// joint j of workgroup jb of a chain's joint blocks (backbone blocks, then
// side-chain blocks); false past the end
__device__ __forceinline__ bool joint_of_block(const ChainDev *cd, int jb, int tid, int *j)
{
    if (jb >= cd->n_bb_blocks) {
        const int jc = (jb - cd->n_bb_blocks) * JOINT_BLOCK + tid;
        *j = cd->n_joints + jc;
        return jc < cd->n_chi;
    }
    *j = jb * JOINT_BLOCK + tid;
    return *j < cd->n_joints;
}

// angle into (-pi, pi]; an angle already inside comes back unchanged
__device__ __forceinline__ double wrap_angle(double t)
{
    t -= 2.0 * PI_D * floor((t + PI_D) / (2.0 * PI_D));
    return t <= -PI_D ? t + 2.0 * PI_D : t;
}

// MC_RESET: the chain re-boots from its current angles (positions, grid),
// with no convergence test or iteration limit, so that every descent runs its
// full length.  MC_PROPOSE: angles = wrap(accepted + delta of this trial) on
// the free joints, then the same re-boot.  A chain with a failure status is
// left alone.
__global__ __launch_bounds__(JOINT_BLOCK) void k_mc_propose(Batch bt, int mode, const double *__restrict__ delta,
                                                             const int64_t *__restrict__ delta_off, int trial)
{
    const int c = find_block_owner(bt.jblk_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    ChainStats *st = cd->stats;
    if (st->status != 0) return;
    const int jb = blockIdx.x - bt.jblk_off[c];
    if (jb == 0 && threadIdx.x == 0) {
        st->need_grid = 1;
        st->pending_post = 0;
        st->post_bad = 0;
        st->converged = 0;
        st->tol = 0.0;
        st->iter_limit = INT64_MAX;
        st->run = 1;
        st->active = 1;
    }
    int j;
    if (mode != MC_PROPOSE || !joint_of_block(cd, jb, threadIdx.x, &j)) return;
    const int Jt = cd->n_joints + cd->n_chi;
    const double a = cd->mc_theta[j];
    cd->theta[j] = cd->mask[j] ? wrap_angle(a + delta[delta_off[c] + (int64_t)trial * Jt + j]) : a;
}

// One thread per chain, after the torque kernel has reduced the energies of
// the last evaluation.  MC_INIT takes the state as the accepted and lowest
// one; MC_TRIAL accepts it when E <= E_acc or u < exp(-(E - E_acc)/kT).  The
// pending step of the last evaluation is discarded either way.
__global__ void k_mc_decide(Batch bt, int mode, const double *__restrict__ u, int n_trials, int trial, double kT)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= bt.n_chains) return;
    const ChainDev *cd = bt.table[c];
    ChainStats *st = cd->stats;
    // the energy of the chain's terms (bits 1 Coulomb, 2 Lennard-Jones, 4 solvation)
    double e = 0.0;
    if (cd->terms & 1) e += st->e_elec;
    if (cd->terms & 2) e += st->e_vdw;
    if (cd->terms & 4) e += st->e_cav;
    if (st->status == 0 && (st->post_bad || !isfinite(e))) st->status = -4;
    const int ok = st->status == 0;
    int acc = 0, best = 0;
    if (mode == MC_INIT) {
        // taken even after a failure, so that the accepted angles are defined
        acc = best = 1;
        st->mc_e_start = st->mc_e_acc = st->mc_e_best = e;
        st->mc_trials = st->mc_accepted = 0;
    } else if (ok) {
        const double de = e - st->mc_e_acc;
        acc = de <= 0.0 || (kT > 0.0 && u[(int64_t)c * n_trials + trial] < exp(-de / kT));
        best = e < st->mc_e_best;
        if (acc) st->mc_e_acc = e;
        if (best) st->mc_e_best = e;
        st->mc_trials += 1;
        st->mc_accepted += acc;
    }
    st->mc_acc = acc;
    st->mc_best = best;
    st->pending_post = 0;
    st->need_grid = 1;
    st->active = ok;
    st->run = ok;
}

// Joint blocks: the lowest and accepted angles take the trial's angles as
// decided; a rejected trial returns the chain to the accepted angles.
__global__ __launch_bounds__(JOINT_BLOCK) void k_mc_apply(Batch bt)
{
    const int c = find_block_owner(bt.jblk_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    const ChainStats *st = cd->stats;
    int j;
    if (!joint_of_block(cd, blockIdx.x - bt.jblk_off[c], threadIdx.x, &j)) return;
    const int Jt = cd->n_joints + cd->n_chi;
    const double p = cd->theta[j];
    if (st->mc_best) cd->mc_theta[Jt + j] = p;
    if (st->mc_acc) cd->mc_theta[j] = p;
    else cd->theta[j] = cd->mc_theta[j];
}

// New angles for every chain of the batch from one device array (chain c's
// J_c angles at theta_off[c]), wrapped into (-pi, pi]; each chain restarts
// like a freshly built one (flags cleared, positions and grid anew).
__global__ __launch_bounds__(JOINT_BLOCK) void k_set_theta(Batch bt, const double *__restrict__ theta,
                                                            const int64_t *__restrict__ theta_off)
{
    const int c = find_block_owner(bt.jblk_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    const int jb = blockIdx.x - bt.jblk_off[c];
    if (jb == 0 && threadIdx.x == 0) {
        ChainStats *st = cd->stats;
        st->converged = 0;
        st->status = 0;
        st->nbr_overflow = 0;
        st->need_grid = 1;
        st->pending_post = 0;
        st->post_bad = 0;
        st->grid_bad = 0;
        st->run = 1;
        st->active = 1;
    }
    int j;
    if (!joint_of_block(cd, jb, threadIdx.x, &j)) return;
    cd->theta[j] = wrap_angle(theta[theta_off[c] + j]);
}

// ---------------------------------------------------------------------------
// cell list: exclusive scan of the counts, counting-sort scatter, stable
// order inside each cell, gather into cell order
// ---------------------------------------------------------------------------
// Chunk offsets of the chain's current grid, block-wide: s_off[b] = number of
// atoms in the cells of the chunks before chunk b, for b = 0 .. nb (s_off[nb]:
// all atoms).  The cell start of cell c is cell_local[c] + s_off[c / SCAN_CHUNK].
__device__ void chunk_offsets(const ChainDev *cd, int nc, int *s_off, int *s_int)
{
    const int nb = (nc + SCAN_CHUNK - 1) / SCAN_CHUNK;
    const int tid = threadIdx.x, per = (nb + blockDim.x - 1) / blockDim.x;
    int loc = 0;
    for (int k = 0; k < per; ++k) {
        const int b = tid * per + k;
        if (b < nb) loc += cd->scan_part[b];
    }
    int total = 0;
    int run = block_excl_scan(loc, s_int, &total);
    for (int k = 0; k < per; ++k) {
        const int b = tid * per + k;
        if (b < nb) {
            s_off[b] = run;
            run += cd->scan_part[b];
        }
    }
    if (tid == 0) s_off[nb] = total;
    __syncthreads();
}

// Slot of atom a in the cell-ordered arrays: the counting-sort scatter placed
// the atoms of a cell in the order of their count atomics; the stable slot is
// the number of atoms of the cell with a smaller index, so everything
// downstream is deterministic.  Gathers position and parameters into that
// slot; w holds the atom index in its low and the atom's residue in its high
// 32 bits (read as integers only).  Returns the rank.
__device__ __forceinline__ int place_sorted(const ChainDev *cd, const int *ids, int a, int b, int e)
{
    // the cell's members four at a time, every load issued before any is
    // compared (indices clamped into the cell, which holds a itself, e > b)
    int rank = 0;
    for (int s = b; s < e; s += 4) {
        int v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = ids[min(s + k, e - 1)];
#pragma unroll
        for (int k = 0; k < 4; ++k) rank += (s + k < e && v[k] < a) ? 1 : 0;
    }
    const int pos = b + rank;
    const double4 r = cd->r[a];
    cd->s_idx[pos] = a;
    cd->s_r[pos] = make_double4(r.x, r.y, r.z, __longlong_as_double((long long)a | ((long long)(a / APR) << 32)));
    cd->s_p[pos] = cd->aparam[a];
    return rank;
}

// k_cellscan: one workgroup per chunk of SCAN_CHUNK cells of each chain's
// capacity (chunks past the current grid return at once): the exclusive scan
// of the counts inside the chunk, and the chunk's total.  Each thread takes
// four consecutive cells as one 16-byte load (the capacity is a multiple of
// 8 cells, so a load that starts inside the grid stays inside the array),
// scans them in registers, and the block scans the thread totals.  The chunk
// offsets are added by the scatter and rank kernels; k_rank writes the final
// starts.
__global__ __launch_bounds__(CHAIN_THREADS) void k_cellscan(Batch bt)
{
    static_assert(SCAN_CHUNK == 4 * CHAIN_THREADS, "four cells per thread");
    const int c = find_block_owner(bt.scan_off, bt.n_chains, blockIdx.x);
    const ChainDev *cd = bt.table[c];
    if (!running(cd->stats)) return;
    const int b = blockIdx.x - bt.scan_off[c];
    const int nc = cd->grid->n_cells, c0 = b * SCAN_CHUNK;
    if (c0 >= nc) return;
    __shared__ int s_int[CHAIN_THREADS / WAVE];
    const int m = min(SCAN_CHUNK, nc - c0), i0 = 4 * (int)threadIdx.x;
    int4 v = make_int4(0, 0, 0, 0);
    if (i0 < m) {
        v = *reinterpret_cast<const int4 *>(cd->cell_count + c0 + i0);
        if (i0 + 1 >= m) v.y = 0;
        if (i0 + 2 >= m) v.z = 0;
        if (i0 + 3 >= m) v.w = 0;
    }
    int total = 0;
    const int run = block_excl_scan(v.x + v.y + v.z + v.w, s_int, &total);
    const int4 o = make_int4(run, run + v.x, run + v.x + v.y, run + v.x + v.y + v.z);
    int *__restrict__ local = cd->cell_local + c0 + i0;
    if (i0 + 3 < m) {
        *reinterpret_cast<int4 *>(local) = o;
    } else if (i0 < m) {
        local[0] = o.x;
        if (i0 + 1 < m) local[1] = o.y;
        if (i0 + 2 < m) local[2] = o.z;
    }
    if (threadIdx.x == 0) cd->scan_part[b] = total;
}

// k_scatter and k_rank: one thread per atom; the dynamic LDS holds the chunk
// offsets (SCAN_MAX_CHUNKS + 1 ints at most).
__global__ __launch_bounds__(ATOM_BLOCK) void k_scatter(Batch bt)
{
    extern __shared__ int s_off[];
    __shared__ int s_int[ATOM_BLOCK / WAVE];
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    const ChainDev *cd = bt.table[c];
    if (!running(cd->stats)) return;
    chunk_offsets(cd, cd->grid->n_cells, s_off, s_int);
    const int a = (blockIdx.x - bt.blk_off[c]) * ATOM_BLOCK + threadIdx.x;
    if (a >= cd->n_atoms) return;
    const int key = cd->cell_key[a];
    const int start = cd->cell_local[key] + s_off[key / SCAN_CHUNK];
    cd->s_tmp[start + cd->s_idx[a]] = a;
}

__global__ __launch_bounds__(ATOM_BLOCK) void k_rank(Batch bt)
{
    extern __shared__ int s_off[];
    __shared__ int s_int[ATOM_BLOCK / WAVE];
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    const ChainDev *cd = bt.table[c];
    if (!running(cd->stats)) return;
    const int nc = cd->grid->n_cells, nb = (nc + SCAN_CHUNK - 1) / SCAN_CHUNK;
    chunk_offsets(cd, nc, s_off, s_int);
    // the final cell starts (nc + 1 of them), a slice per workgroup of the chain
    const int lb = blockIdx.x - bt.blk_off[c], nblk = bt.blk_off[c + 1] - bt.blk_off[c];
    const int per = (nc + 1 + nblk - 1) / nblk, i1 = min(nc + 1, (lb + 1) * per);
    {
        // four cells per thread per step, the loads issued before the stores
        // (indices clamped into the grid, which has at least one cell)
        const int *__restrict__ loc = cd->cell_local;
        int *__restrict__ start = cd->cell_start;
        for (int i = lb * per + (int)threadIdx.x; i < i1; i += 4 * ATOM_BLOCK) {
            int v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = loc[min(i + k * ATOM_BLOCK, nc - 1)];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int j = i + k * ATOM_BLOCK;
                if (j < i1) start[j] = j < nc ? v[k] + s_off[j / SCAN_CHUNK] : s_off[nb];
            }
        }
    }
    const int a = lb * ATOM_BLOCK + threadIdx.x;
    if (a >= cd->n_atoms) return;
    const int key = cd->cell_key[a];
    const int b = cd->cell_local[key] + s_off[key / SCAN_CHUNK];
    const int e = key + 1 < nc ? cd->cell_local[key + 1] + s_off[(key + 1) / SCAN_CHUNK] : s_off[nb];
    // the first atom of each cell returns its count to zero for the next iteration
    if (place_sorted(cd, cd->s_tmp, a, b, e) == 0) cd->cell_count[key] = 0;
}

// Loads, stores and atomics through a pointer of unknown address space are
// flat instructions, which count against the LDS counter as well as the
// vector-memory one: every LDS wait then also waits for them.  The device
// arrays of the force kernel are all in global memory, and it reaches them
// through these global-address-space views (plain pointers in the host
// pass, which only checks the device code).
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T> using gptr = __attribute__((address_space(1))) T *;
#else
template <typename T> using gptr = T *;
#endif
template <typename T> __device__ __forceinline__ gptr<T> glob(T *p) { return (gptr<T>)p; }
using CDev = gptr<const ChainDev>;
// fixed-point accumulation of the solvation force
__device__ __forceinline__ void fix_add(gptr<long long> p, long long v)
{
    __hip_atomic_fetch_add((gptr<unsigned long long>)p, (unsigned long long)v, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------
// k_force: Coulomb + LJ + SASA enumeration, one wave per atom
// ---------------------------------------------------------------------------
// A solvation neighbour j of atom i: offset a = r_j - r_i and the threshold c0 =
// (R_i^2 + |a|^2 - R_j^2) / (2 R_i): sample q_k = r_i + R_i Q_k is covered by j iff
// Q_k . a >= c0 (the same test as ||q_k - r_j|| <= R_j).
template <typename Real>
struct NbrEntry {
    Real ax, ay, az, c0;
};

// Squared distance and cap threshold of a candidate, with the fused steps
// written out: every path and launch shape that takes them rounds alike.
__device__ __forceinline__ double dist2(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return fma(dz, dz, fma(dy, dy, dx * dx));
}
// set bits of m in the lanes below this one (the hardware's masked bit count)
__device__ __forceinline__ int count_below(unsigned long long m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}
__device__ __forceinline__ double cap_c0(double roff_i, double d2, double rj, double inv_2roff)
{
#pragma clang fp contract(off)
    return fma(-rj, rj, fma(roff_i, roff_i, d2)) * inv_2roff;
}

constexpr int SPL = 4;                              // samples per lane in one pass: passes of 256 samples
// Neighbours whose cap on the offset sphere is large (cosine of its angular
// radius, c0/|a|, below CAP_SPLIT) lead the list: step 1 then reaches two
// overlappers for every sample of a slot early and stops there.
constexpr double CAP_SPLIT = 0.6;
// Launch shapes of the force kernel (kcm_set_force_variant): candidates each
// lane loads per trip of the candidate loop (CPT), the neighbours step 1
// reads as one block before it checks the slots' saturation (SATB), and the
// order of the atoms over the workgroups: cell order, or XCD-aware (the
// workgroups go to the 8 XCDs in turn; XCD x takes the x-th contiguous eighth
// of the cell-ordered atoms, so that its L2 serves one region of space).
// Every shape visits the candidates and appends the neighbours in the same
// order, and takes the same decisions: the results are the same bit for bit.
struct ForceShape {
    int cpt, satb;
    bool xcd;
};
constexpr ForceShape FORCE_SHAPES[] = {{2, 4, false}, {1, 4, false}, {1, 4, true}, {2, 4, true}};
constexpr int N_XCD = 8;
constexpr int NSLOT = (MAX_NBR + WAVE - 1) / WAVE;  // neighbours per lane in step 2
// Step-1 count of a sample: acc = (covering neighbours << ACC_SHIFT) + (sum of
// their slots), so acc >> ACC_SHIFT == 1 leaves the single overlapper in the
// low bits; slots below MAX_NBR keep the slot sum below 2^ACC_SHIFT.
constexpr int ACC_SHIFT = 17;
// After the first COMPACT_AT neighbours of the list, the samples of a pass
// that can still change (fewer than two overlappers so far, or a test inside
// the FP32 band) move to the leading slots, in sample order, and the others
// count as covered; the later blocks test only the slots that hold them.
// Each moves as one word in the unused end of the neighbour list: acc (below
// 2^STAGE_K: at most COMPACT_AT overlappers), its sample within the pass, and
// its band flag.
constexpr int COMPACT_AT = 16;
constexpr int STAGE_K = 22;
static_assert(COMPACT_AT * ((1 << ACC_SHIFT) + COMPACT_AT) < (1 << STAGE_K), "staged count field");
static_assert(WAVE * SPL <= 256 && STAGE_K + 8 < 31, "staged sample field");
static_assert(MAX_NBR * (MAX_NBR - 1) / 2 < (1 << ACC_SHIFT), "slot sum must stay below the count field");
static_assert(MAX_NBR * 2 < (1 << (31 - ACC_SHIFT)), "count field must not overflow");
static_assert((2 * MAX_REACH + 1) * (2 * MAX_REACH + 1) <= WAVE, "stencil rows must fit one wave");
// Net events of one neighbour and axis lie in [-N, N] with N < 2^15 samples:
// axes 0 and 1 share a word as two halves biased by 2^15 (no carry or borrow
// crosses the halves), axis 2 has a word of its own.
constexpr int EV_BIAS = 0x8000;
constexpr int EV_INIT = EV_BIAS | (EV_BIAS << 16);

__device__ __forceinline__ float bcast(float x, int l)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ __forceinline__ double bcast(double x, int l)
{
    const long long b = __double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// a * b + c for a, b below 2^24 (b wave-uniform) as one full-rate 24-bit
// multiply-add; the compiler otherwise may pick the quarter-rate 32-bit
// multiply when it cannot bound b.
__device__ __forceinline__ int mad_u24(int a, int b, int c)
{
    int r;
    asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
    return r;
}

// Step-1 code of four FP32 tests t0..t3 of one sample against the neighbours
// of a block: the sum of 32 + q over the tests with t_q >= 0.  Two byte
// permutes gather the four sign bits as bytes (0xff for a negative test,
// selectors 9 and 11 replicate the top bit of the low and the high source
// word), and a signed dot product with the bytes 32..35 subtracts 32 + q for
// each negative test from the sum over all four (134).  A test of exactly -0
// counts as uncovered here; |t| = 0 lies in the FP32 band, so its sample is
// decided again in FP64.
__device__ __forceinline__ int block_code(float t0, float t1, float t2, float t3)
{
    const unsigned lo = __builtin_amdgcn_perm(__float_as_uint(t1), __float_as_uint(t0), 0x0c0c0b09u);
    const unsigned hi = __builtin_amdgcn_perm(__float_as_uint(t3), __float_as_uint(t2), 0x0b090c0cu);
    constexpr int ALL = 4 * 32 + 0 + 1 + 2 + 3;
    return __builtin_amdgcn_sdot4((int)(lo | hi), 0x23222120, ALL, false);
}

// FP64 decision in absolute coordinates: is sample k of atom i covered by the
// offset sphere of atom aj, shifted by delta_r along axis s (s < 0: not
// shifted)?
__device__ __forceinline__ bool cover_exact(CDev cd, const double4 &ri, double roff_i, int k, int aj, int s)
{
    const double4 q = glob(cd->q64)[k];
    const double qx = ri.x + roff_i * q.x, qy = ri.y + roff_i * q.y, qz = ri.z + roff_i * q.z;
    double4 c = glob(cd->r)[aj];
    if (s == 0) c.x += cd->delta_r;
    if (s == 1) c.y += cd->delta_r;
    if (s == 2) c.z += cd->delta_r;
    const double rj = glob(cd->aparam)[aj].w;
    const double dx = qx - c.x, dy = qy - c.y, dz = qz - c.z;
    return dx * dx + dy * dy + dz * dz - rj * rj <= 0.0;
}

// Coverage by a displaced neighbour, v = (tested quantity) with threshold 0;
// the mixed form decides again in FP64 inside the band.
template <typename Real, bool MIXED>
__device__ __forceinline__ bool test_cover(Real v, CDev cd, const double4 &ri, double roff_i, int k, int aj, int s)
{
    bool hit = v >= (Real)0;
    if (MIXED) {
        if (fabsf((float)v) <= MIXED_BAND) hit = cover_exact(cd, ri, roff_i, k, aj, s);
    }
    return hit;
}

// The three displaced tests of one (sample, neighbour) pair are decided in
// the form's precision first; the mixed form then takes every test inside the
// band again in FP64, the three behind one branch.  band3: is any of them in
// the band; redo: the FP32 decision minus the FP64 one for a test in the band
// (0 outside it), the correction to a count of covered tests.
__device__ __forceinline__ bool band3(float v0, float v1, float v2)
{
    return fminf(fabsf(v0), fminf(fabsf(v1), fabsf(v2))) <= MIXED_BAND;
}
__device__ __forceinline__ int redo(float v, CDev cd, const double4 &ri, double roff_i, int k, int aj, int s)
{
    if (fabsf(v) > MIXED_BAND) return 0;
    return (v >= 0.0f ? 1 : 0) - (cover_exact(cd, ri, roff_i, k, aj, s) ? 1 : 0);
}

template <typename Real>
__device__ __forceinline__ void load_q(CDev cd, int k, Real &x, Real &y, Real &z)
{
    if (sizeof(Real) == 4) {
        const float4 q = glob(cd->q32)[k];
        x = (Real)q.x; y = (Real)q.y; z = (Real)q.z;
    } else {
        const double4 q = glob(cd->q64)[k];
        x = (Real)q.x; y = (Real)q.y; z = (Real)q.z;
    }
}

// One lane's Coulomb + LJ sums over its candidates (the stencil rows of the
// calling wave), all in FP64.  Called, out of line, for an atom whose FP32
// pair terms left the FP32 range: atoms a few hundredths of an angstrom apart
// drive (D/d)^12 and the force past it.  Same candidates, cutoff decisions and
// weights as the force kernel (eqs 02, 03).
struct PairSums {
    double f[3];
    double e[2];
};
__device__ __noinline__ PairSums pair_terms_fp64(CDev cd, int si, int off, int rbase, int T, int nrows,
                                                 int res_i, uint32_t m12, uint32_t m13, uint32_t m14, int terms)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const double4 ri = glob(cd->s_r)[si];
    const double4 pa = glob(cd->s_p)[si];
    const double cut2 = cd->cutoff * cd->cutoff;
    const bool do_elec = terms & 1, do_vdw = terms & 2;
    PairSums out = {{0.0, 0.0, 0.0}, {0.0, 0.0}};
#pragma unroll 1
    for (int kb = 0; kb < T; kb += WAVE) {
        const int k = kb + lane;
        int lo = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const int t = lo + step;
            const int o = __shfl(off, t & (WAVE - 1), WAVE);
            if (t < nrows && o <= k) lo = t;
        }
        int sj = __shfl(rbase, lo, WAVE) + k;
        const bool ok = k < T && sj != si;
        if (k >= T) sj = si;
        const double4 rj = glob(cd->s_r)[sj];
        const double4 pj = glob(cd->s_p)[sj];
        const double ddx = rj.x - ri.x, ddy = rj.y - ri.y, ddz = rj.z - ri.z;
        const double d2 = dist2(ddx, ddy, ddz);
        if (!(ok && d2 <= cut2)) continue;
        const long long wj = __double_as_longlong(rj.w);
        const int aj = (int)wj, res_j = (int)(wj >> 32), dres = res_j - res_i;
        double we = do_elec ? 1.0 : 0.0, wv = do_vdw ? 1.0 : 0.0;
        if (dres >= -1 && dres <= 1) {
            const uint32_t bit = 1u << ((dres + 1) * APR + (aj - res_j * APR));
            if (m12 & bit) { we = 0; wv = 0; }
            else if (m13 & bit) { we *= cd->w13; wv *= cd->w13; }
            else if (m14 & bit) { we *= cd->w14e; wv *= cd->w14v; }
        }
        if (we == 0.0 && wv == 0.0) continue;
        const double inv2 = 1.0 / d2;
        const double eel = we * cd->coulomb * pa.x * pj.x * inv2;
        const double D = pa.y + pj.y;
        const double s2 = D * D * inv2, s6 = s2 * s2 * s2, s12 = s6 * s6;
        const double eij = pa.z * pj.z;
        const double fsc = (2.0 * eel + 12.0 * wv * eij * (s12 - s6)) * inv2;
        out.f[0] -= fsc * ddx;
        out.f[1] -= fsc * ddy;
        out.f[2] -= fsc * ddz;
        out.e[0] += eel;
        out.e[1] += wv * eij * (s12 - 2.0 * s6);
    }
    return out;
}

// Solvation of one atom with more neighbours than the LDS list holds (dense
// self-overlaps of random starts).  Called, out of line, by the force kernel's
// wave for that atom; the common path keeps its list in LDS in one piece.
// The neighbours are numbered in candidate order, as the kernel numbers them,
// and taken in chunks of MAX_NBR, each enumerated again from the candidates
// (the wave's stencil rows: off, rbase, nrows, T) into the kernel's LDS
// arrays when needed.  Step 1 runs over every chunk; a sample's count
// saturates at 2 (only 0, 1 and more matter) and keeps the single
// overlapper's number.  Step 2 and the event scatter go chunk by chunk.  The
// decisions are those of one list, so the results are the same.
struct ChunkedSasa {
    int ncov;                 // covered samples of this lane
    int own[3];               // this lane's share of the atom's own net events per axis
};
struct ChunkArgs {
    int si, off, rbase, nrows, T, nn;
};
template <typename Real>
__device__ __noinline__ ChunkedSasa sasa_chunked(CDev cd, const ChunkArgs c, NbrEntry<Real> *s_nbr,
                                                 int *s_nbr_a, unsigned *s_ev01, int *s_ev2)
{
    constexpr bool MIXED = sizeof(Real) == 4;
    const int lane = threadIdx.x & (WAVE - 1);
    // the atom's quantities, read again rather than passed (the call then
    // keeps few of the kernel's registers live)
    struct {
        int si, off, rbase, nrows, T, nn, N;
        double4 ri;
        double roff_i, inv_2roff, dr;
        long long qf;
    } a;
    a.si = c.si; a.off = c.off; a.rbase = c.rbase; a.nrows = c.nrows; a.T = c.T; a.nn = c.nn;
    a.N = cd->n_samples;
    a.ri = glob(cd->s_r)[c.si];
    a.roff_i = glob(cd->s_p)[c.si].w;
    a.inv_2roff = 0.5 / a.roff_i;
    a.dr = cd->delta_r;
    a.qf = glob(cd->qfix)[(int)__double_as_longlong(a.ri.w)];
    const Real drr = (Real)a.dr, kq = (Real)(a.dr * a.dr / (2.0 * a.roff_i)), k1 = (Real)(a.dr / a.roff_i);
    const Real guard = MIXED ? (Real)(2.0f * MIXED_BAND) : (Real)1e-9;
    ChunkedSasa out = {0, {0, 0, 0}};

    // neighbours numbered [lo, lo + len) into LDS positions 0 .. len-1
    auto enum_window = [&](int lo, int len) {
        int nb = 0;
#pragma unroll 1
        for (int kb = 0; kb < a.T; kb += WAVE) {
            const int k = kb + lane;
            int r = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int t = r + step;
                const int o = __shfl(a.off, t & (WAVE - 1), WAVE);
                if (t < a.nrows && o <= k) r = t;
            }
            int sj = __shfl(a.rbase, r, WAVE) + k;
            const bool valid = k < a.T && sj != a.si;
            if (k >= a.T) sj = a.si;
            const double4 rj = glob(cd->s_r)[sj];
            const double4 pj = glob(cd->s_p)[sj];
            const double ddx = rj.x - a.ri.x, ddy = rj.y - a.ri.y, ddz = rj.z - a.ri.z;
            const double d2 = dist2(ddx, ddy, ddz);
            const double lim = a.roff_i + pj.w + a.dr;
            const bool in_cav = valid && d2 <= lim * lim;
            const unsigned long long m = __ballot(in_cav);
            if (in_cav) {
                const int pos = nb + count_below(m) - lo;
                if (pos >= 0 && pos < len) {
                    NbrEntry<Real> e;
                    e.ax = (Real)ddx; e.ay = (Real)ddy; e.az = (Real)ddz;
                    e.c0 = (Real)cap_c0(a.roff_i, d2, pj.w, a.inv_2roff);
                    s_nbr[pos] = e;
                    s_nbr_a[pos] = (int)__double_as_longlong(rj.w);
                }
            }
            nb += __popcll(m);
        }
    };

#pragma unroll 1
    for (int kb = 0; kb < a.N; kb += WAVE * SPL) {
        Real Qx[SPL], Qy[SPL], Qz[SPL];
        int cnt[SPL], who[SPL];
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
            const int k = kb + lane + WAVE * i;
            Qx[i] = Qy[i] = Qz[i] = (Real)0;
            if (k < a.N) load_q<Real>(cd, k, Qx[i], Qy[i], Qz[i]);
            cnt[i] = who[i] = 0;
        }
        // step 1 over every chunk
        for (int lo = 0; lo < a.nn; lo += MAX_NBR) {
            const int len = min(a.nn - lo, MAX_NBR);
            __syncthreads();
            enum_window(lo, len);
            __syncthreads();
            int acc[SPL];
            Real amin[SPL];
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                acc[i] = 0;
                amin[i] = (Real)1e30;
            }
            for (int u = 0; u < len; ++u) {
                const NbrEntry<Real> e = s_nbr[u];
                const int inc = (1 << ACC_SHIFT) + u;
#pragma unroll
                for (int i = 0; i < SPL; ++i) {
                    const Real t = fma(Qz[i], e.az, fma(Qy[i], e.ay, fma(Qx[i], e.ax, -e.c0)));
                    acc[i] += (t >= (Real)0) ? inc : 0;
                    if (MIXED) amin[i] = fmin(amin[i], fabs(t));
                }
            }
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                if (MIXED) {
                    // a test within the band of its threshold: the whole wave
                    // recounts that sample in FP64, one lane per neighbour
                    unsigned long long bm = __ballot(kb + lane + WAVE * i < a.N && amin[i] <= (Real)MIXED_BAND);
                    while (bm) {
                        const int l = __ffsll((long long)bm) - 1;
                        bm &= bm - 1;
                        const int kl = kb + l + WAVE * i;
                        int part = 0;
                        for (int u = lane; u < len; u += WAVE)
                            if (cover_exact(cd, a.ri, a.roff_i, kl, s_nbr_a[u], -1)) part += (1 << ACC_SHIFT) + u;
                        part = wave_sum_i(part);
                        if (lane == l) acc[i] = part;
                    }
                }
                const int cc = acc[i] >> ACC_SHIFT;
                if (cc == 1) who[i] = lo + (acc[i] & ((1 << ACC_SHIFT) - 1));
                cnt[i] = min(cnt[i] + cc, 2);
            }
        }
#pragma unroll
        for (int i = 0; i < SPL; ++i)
            if (kb + lane + WAVE * i < a.N && cnt[i] >= 1) ++out.ncov;
        // step 2 and the events, chunk by chunk
        for (int lo = 0; lo < a.nn; lo += MAX_NBR) {
            const int len = min(a.nn - lo, MAX_NBR);
            __syncthreads();
            enum_window(lo, len);
            for (int u = lane; u < len; u += WAVE) {
                s_ev01[u] = EV_INIT;
                s_ev2[u] = 0;
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                const int k = kb + lane + WAVE * i;
                const bool valid = k < a.N;
                if (valid && cnt[i] == 1 && who[i] >= lo && who[i] < lo + len) {
                    // critically overlapped: only the overlapper's shifted copies can expose it
                    const int u = who[i] - lo;
                    const NbrEntry<Real> e = s_nbr[u];
                    const int aj = s_nbr_a[u];
                    const Real base = Qx[i] * e.ax + Qy[i] * e.ay + Qz[i] * e.az - e.c0 - kq;
                    const Real span = drr + k1 * fmax(fabs(e.ax), fmax(fabs(e.ay), fabs(e.az)));
                    if (base - span <= guard) {
                        unsigned inc01 = 0;
                        if (!test_cover<Real, MIXED>(base + drr * Qx[i] - k1 * e.ax, cd, a.ri, a.roff_i, k, aj, 0)) inc01 += 1u;
                        if (!test_cover<Real, MIXED>(base + drr * Qy[i] - k1 * e.ay, cd, a.ri, a.roff_i, k, aj, 1)) inc01 += 1u << 16;
                        if (inc01) atomicAdd(&s_ev01[u], inc01);
                        if (!test_cover<Real, MIXED>(base + drr * Qz[i] - k1 * e.az, cd, a.ri, a.roff_i, k, aj, 2)) atomicAdd(&s_ev2[u], 1);
                    }
                }
                // exposed samples: one lane per neighbour, the samples broadcast
                const unsigned long long em0 = __ballot(valid && cnt[i] == 0);
                if (!em0) continue;
                for (int v = 0; WAVE * v < len; ++v) {
                    const int u = lane + WAVE * v;
                    const bool own = u < len;
                    const NbrEntry<Real> e = s_nbr[own ? u : 0];
                    const int aj = s_nbr_a[own ? u : 0];
                    const Real lim = -(drr + k1 * fmax(fabs(e.ax), fmax(fabs(e.ay), fabs(e.az)))) - guard;
                    int d0 = 0, d1 = 0, d2 = 0;
                    unsigned long long em = em0;
                    while (em) {
                        const int l = __ffsll((long long)em) - 1;
                        em &= em - 1;
                        const Real qx = bcast(Qx[i], l), qy = bcast(Qy[i], l), qz = bcast(Qz[i], l);
                        const Real base = qx * e.ax + qy * e.ay + qz * e.az - e.c0 - kq;
                        if (own && base >= lim) {
                            const int kx = kb + l + WAVE * i;
                            if (test_cover<Real, MIXED>(base + drr * qx - k1 * e.ax, cd, a.ri, a.roff_i, kx, aj, 0)) --d0;
                            if (test_cover<Real, MIXED>(base + drr * qy - k1 * e.ay, cd, a.ri, a.roff_i, kx, aj, 1)) --d1;
                            if (test_cover<Real, MIXED>(base + drr * qz - k1 * e.az, cd, a.ri, a.roff_i, kx, aj, 2)) --d2;
                        }
                    }
                    const unsigned dec01 = (unsigned)d0 + ((unsigned)d1 << 16);
                    if (own && dec01) atomicAdd(&s_ev01[u], dec01);
                    if (own && d2) atomicAdd(&s_ev2[u], d2);
                }
            }
            __syncthreads();
            // eq F_cav_patch: atom i gains G0_i ev / (N dr) per axis, neighbour j the opposite
            for (int u = lane; u < len; u += WAVE) {
                const unsigned w01 = s_ev01[u];
                const int e0 = (int)(w01 & 0xffffu) - EV_BIAS, e1 = (int)(w01 >> 16) - EV_BIAS, e2 = s_ev2[u];
                const int aj = s_nbr_a[u];
                const int ev[3] = {e0, e1, e2};
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    if (!ev[x]) continue;
                    out.own[x] += ev[x];
                    fix_add(&glob(cd->f_cav)[3 * aj + x], (-(long long)ev[x] * a.qf));
                }
            }
        }
    }
    return out;
}

// Mixed form: six waves per SIMD (80 registers, the 6,720-byte LDS list), which
// hides the latency of the candidate loads and LDS reads better than four
// waves with room to spare (3.06 against 3.39 ms on the 256-chain batch);
// seven spill in the hot loops.  The FP64 form: four (127 registers; its
// 10,560-byte list allows 15 waves per CU).
template <typename Real, int CPT, int SAT_CHECK, bool XCD>
__global__ __launch_bounds__(WAVE, sizeof(Real) == 4 ? 6 : 4) void k_force(Batch bt)
{
    static_assert(SAT_CHECK * (SAT_CHECK - 1) / 2 < 32 && 32 + SAT_CHECK <= 64, "block code of step 1");
    constexpr bool MIXED = sizeof(Real) == 4;
    __shared__ NbrEntry<Real> s_nbr[MAX_NBR];
    __shared__ int s_nbr_a[MAX_NBR];
    __shared__ __align__(8) unsigned s_ev01[MAX_NBR];  // net events of each neighbour, axes 0 and 1 (biased halves)
    __shared__ int s_ev2[MAX_NBR];                     // and axis 2

    int atom = blockIdx.x;
    if (XCD) {
        const int nq = bt.total_atoms / N_XCD, nr = bt.total_atoms % N_XCD;
        const int x = blockIdx.x % N_XCD, k = blockIdx.x / N_XCD;
        atom = x * nq + min(x, nr) + k;
    }
    const int c = find_block_owner(bt.atom_off, bt.n_chains, atom);
    const CDev cd = glob(glob(bt.table)[c]);
    if (!running(cd->stats)) return;
    const int si = atom - bt.atom_off[c];
    const int lane = threadIdx.x;

    const Grid g = *glob(cd->grid);
    const double4 ri = glob(cd->s_r)[si];
    const double4 pi = glob(cd->s_p)[si];
    const int ai = (int)__double_as_longlong(ri.w);
    const int dxn = g.dims[0], dyn = g.dims[1], dzn = g.dims[2];
    // the atom's cell, by the expression that sorted it (no key decoding)
    const int cx = min(max((int)floor((ri.x - g.origin[0]) * g.inv_cell), 0), dxn - 1);
    const int cy = min(max((int)floor((ri.y - g.origin[1]) * g.inv_cell), 0), dyn - 1);
    const int cz = min(max((int)floor((ri.z - g.origin[2]) * g.inv_cell), 0), dzn - 1);
    const int R = g.reach, side = 2 * R + 1, nrows = side * side;
    // lane = row_z * side + row_y; side <= 8 and lane < 64 keep the FP32
    // quotient at least 1/16 away from an integer, far above its rounding
    const int row_z = (int)(((float)lane + 0.5f) * __builtin_amdgcn_rcpf((float)side));
    const int row_y = lane - row_z * side;

    // stencil rows, one per lane: for each (dy, dz) one contiguous run of
    // cells along x, i.e. one contiguous run of the cell-ordered atoms.  The
    // run keeps only the cells that can hold an atom within reach of atom i:
    // a row whose y-z slab is farther than the reach is empty, and the x run
    // covers [x_i - ext, x_i + ext] with ext^2 = reach^2 - (y-z distance)^2.
    // Border cells reach to infinity outward (atoms outside the grid are
    // clamped into them); the pad on the reach absorbs rounding.
    int beg = 0, cnt = 0;
    if (lane < nrows) {
        const int y = cy + row_y - R, z = cz + row_z - R;
        if (y >= 0 && y < dyn && z >= 0 && z < dzn) {
            const double reach = g.reach_len + 1e-6;
            const double ylo = y == 0 ? -DBL_MAX : g.origin[1] + y * g.cell;
            const double yhi = y == dyn - 1 ? DBL_MAX : g.origin[1] + (y + 1) * g.cell;
            const double zlo = z == 0 ? -DBL_MAX : g.origin[2] + z * g.cell;
            const double zhi = z == dzn - 1 ? DBL_MAX : g.origin[2] + (z + 1) * g.cell;
            const double gy = fmax(0.0, fmax(ylo - ri.y, ri.y - yhi));
            const double gz = fmax(0.0, fmax(zlo - ri.z, ri.z - zhi));
            const double rest = reach * reach - gy * gy - gz * gz;
            if (rest >= 0.0) {
                const double ext = sqrt(rest);
                const int xa = (int)floor((ri.x - ext - g.origin[0]) * g.inv_cell);
                const int xb = (int)floor((ri.x + ext - g.origin[0]) * g.inv_cell);
                const int xl = max(max(0, cx - R), min(xa, dxn - 1));
                const int xh = min(min(dxn - 1, cx + R), max(xb, 0));
                if (xl <= xh) {
                    const int base = (z * dyn + y) * dxn;
                    beg = glob(cd->cell_start)[base + xl];
                    cnt = glob(cd->cell_start)[base + xh + 1] - beg;
                }
            }
        }
    }
    int off = cnt;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int y = __shfl_up(off, d, WAVE);
        if (lane >= d) off += y;
    }
    const int T = __shfl(off, WAVE - 1, WAVE);
    off -= cnt;                   // first candidate number of this row
    const int rbase = beg - off;  // candidate number k of row t is sorted atom rbase_t + k

    const int terms = cd->terms;
    const bool do_elec = terms & 1, do_vdw = terms & 2, do_cav = terms & 4;
    const bool do_pair = do_elec || do_vdw;
    const double cut2 = cd->cutoff * cd->cutoff;
    const double roff_i = pi.w;
    const double inv_2roff = 0.5 / roff_i;
    const double dr = cd->delta_r;
    const int res_i = ai / APR, slot_i = ai - res_i * APR;
    const Real coul = (Real)cd->coulomb;
    const Real qi = (Real)pi.x, Ri = (Real)pi.y, sei = (Real)pi.z;

    // Bond class of each atom of residues res_i - 1 .. res_i + 1 relative to
    // atom i, two bits per atom (0 none, 1 1-2, 2 1-3, 3 1-4), and the pair
    // weights (elec, vdw) of each class, copied to LDS after the window table
    // below in the event array (free until the candidates are done).
    const unsigned long long cls_word = cd->cls_word[slot_i];
    const int skip_cls = MIXED ? cd->skip_cls32 : cd->skip_cls64;  // bit c: class c adds nothing
    Real *s_wtab = reinterpret_cast<Real *>(s_ev01 + 2 * WAVE);
    if (lane < 8) s_wtab[lane] = MIXED ? (Real)cd->wtab32[lane] : (Real)cd->wtab64[lane];
    __builtin_amdgcn_wave_barrier();

    // Sorted atom of candidate kw + lane, one window of 64 candidates at a
    // time, windows in increasing order.  Each non-empty row starting inside
    // the window leaves (its first candidate number, rbase) at that position
    // of an LDS table; a candidate's row is the last start at or before it,
    // read from the wave's mask of starts, or else the row running on from
    // the previous window.  The table lives in the event array, which is
    // free until the candidates are done; an entry left by an earlier window
    // never matches, since it holds that window's candidate number.
    int2 *s_head = reinterpret_cast<int2 *>(s_ev01);
    s_head[lane] = make_int2(-1, 0);
    int carry = 0;
    auto window_atom = [&](int kw) -> int {
        if (cnt > 0 && off >= kw && off < kw + WAVE) s_head[off - kw] = make_int2(off, rbase);
        __builtin_amdgcn_wave_barrier();
        const int2 h = s_head[lane];
        // the last start at or below this lane: its bit moved to the top
        const unsigned long long m = __ballot(h.x == kw + lane) << (63 - lane);
        const int p = m ? lane - __clzll((long long)m) : lane;
        const int rb = __shfl(h.y, p, WAVE);
        const int base = m ? rb : carry;
        carry = __builtin_amdgcn_readlane(base, WAVE - 1);
        __builtin_amdgcn_wave_barrier();
        return base + kw + lane;
    };

    Real fx = 0, fy = 0, fz = 0;
    double ee = 0.0, evw = 0.0;
    int nn = 0, nfront = 0, nback = 0;
    // one candidate: pair terms into (fx, fy, fz, ee, evw); a solvation
    // neighbour with a large cap is appended at the front of the list, any
    // other at its back (growing down from MAX_NBR - 1), in lane order
    auto visit = [&](bool valid, const double4 &rj, const double4 &pj) {
        // contraction off, the fused steps written out: the loop bodies of
        // all launch shapes round alike
#pragma clang fp contract(off)
        const double ddx = rj.x - ri.x, ddy = rj.y - ri.y, ddz = rj.z - ri.z;
        const double d2 = dist2(ddx, ddy, ddz);
        const int aj = (int)__double_as_longlong(rj.w);
        if (valid && do_pair && d2 <= cut2) {
            // (dres + 1) APR + slot_j, in [0, 3 APR) iff |dres| <= 1
            const int idx = aj - APR * res_i + APR;
            const int cls = (unsigned)idx < 3u * APR ? (int)((cls_word >> (2 * idx)) & 3) : 0;
            if (!((skip_cls >> cls) & 1)) {
                const Real we = s_wtab[2 * cls], wv = s_wtab[2 * cls + 1];
                const Real rx = (Real)ddx, ry = (Real)ddy, rz = (Real)ddz;
                // mixed form: hardware reciprocal (1 ulp), far inside the force tolerance
                const Real inv2 = MIXED ? (Real)__builtin_amdgcn_rcpf((float)d2) : (Real)1 / (Real)d2;
                // eq 02 with eps = k_d d: E = (C/k_d) q_i q_j / d^2
                const Real eel = we * coul * qi * (Real)pj.x * inv2;
                // eq 03: E = eps_ij [(D/d)^12 - 2 (D/d)^6], D = R_i + R_j, eps_ij = sqrt(eps_i eps_j)
                const Real D = Ri + (Real)pj.y;
                const Real s2 = D * D * inv2, s6 = s2 * s2 * s2, s12 = s6 * s6;
                const Real eij = sei * (Real)pj.z;
                const Real elj = wv * eij * fma((Real)-2, s6, s12);
                // |F|/d along r_i - r_j: 2 E_elec/d^2 + 12 eps (s12 - s6)/d^2
                const Real fsc = fma((Real)2, eel, (Real)12 * wv * eij * (s12 - s6)) * inv2;
                fx = fma(-fsc, rx, fx);
                fy = fma(-fsc, ry, fy);
                fz = fma(-fsc, rz, fz);
                ee += (double)eel;
                evw += (double)elj;
            }
        }
        bool in_cav = false, front = false;
        double c0 = 0.0;
        if (do_cav) {
            const double Rj = pj.w;
            const double lim = roff_i + Rj + dr;
            in_cav = valid && d2 <= lim * lim;
            c0 = cap_c0(roff_i, d2, Rj, inv_2roff);
            front = c0 < 0.0 || c0 * c0 < (CAP_SPLIT * CAP_SPLIT) * d2;
        }
        const unsigned long long mf = __ballot(in_cav && front), mb = __ballot(in_cav && !front);
        const int cf = __popcll(mf), cb = __popcll(mb);
        // past the list's capacity nothing more is written: the atom then
        // takes the chunked path, which enumerates its neighbours again
        if (in_cav && nfront + cf + nback + cb <= MAX_NBR) {
            const int pos = front ? nfront + count_below(mf) : MAX_NBR - 1 - nback - count_below(mb);
            NbrEntry<Real> e;
            e.ax = (Real)ddx; e.ay = (Real)ddy; e.az = (Real)ddz;
            e.c0 = (Real)c0;
            s_nbr[pos] = e;
            s_nbr_a[pos] = aj;
        }
        nfront += cf;
        nback += cb;
        nn += cf + cb;
    };

    // CPT candidates per lane per trip, every load issued before any is used.
    // Loads take 32-bit byte offsets from the chain's arrays (n < 2^26 atoms
    // of 32 bytes).
    const gptr<const char> sr = (gptr<const char>)glob(cd->s_r), sp = (gptr<const char>)glob(cd->s_p);
    // The sorted atoms of the next trip are found while this trip's loads are
    // in flight.
    int sj[CPT];
    auto map_trip = [&](int kb) {
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            const int w = window_atom(kb + q * WAVE);  // wave-wide: every lane takes part
            sj[q] = kb + q * WAVE + lane < T ? w : si;
        }
    };
    if (T > 0) map_trip(0);
    for (int kb = 0; kb < T; kb += CPT * WAVE) {
        bool ok[CPT];
        double4 rj[CPT], pj[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
            ok[q] = sj[q] != si;
            const unsigned ob = (unsigned)sj[q] * (unsigned)sizeof(double4);
            rj[q] = *(const gptr<const double4>)(sr + ob);
            pj[q] = *(const gptr<const double4>)(sp + ob);
        }
        if (kb + CPT * WAVE < T) map_trip(kb + CPT * WAVE);
#pragma unroll
        for (int q = 0; q < CPT; ++q) visit(ok[q], rj[q], pj[q]);
    }

    // pair force and energies of atom i (each unordered pair is seen from both ends)
    double pv[5] = {(double)fx, (double)fy, (double)fz, ee, evw};
    const bool overflow = !(isfinite(pv[0]) && isfinite(pv[1]) && isfinite(pv[2]) && isfinite(ee) && isfinite(evw));
    if (MIXED && __any(overflow)) {
        // Atoms a few thousandths of an angstrom apart drive (D/d)^12 and the
        // force past the FP32 range: this atom's pair terms are taken again,
        // all in FP64 (a non-finite result then is a true one)
        const PairSums ps = pair_terms_fp64(cd, si, off, rbase, T, nrows, res_i, cd->m12[slot_i], cd->m13[slot_i],
                                            cd->m14[slot_i], terms);
        pv[0] = ps.f[0]; pv[1] = ps.f[1]; pv[2] = ps.f[2]; pv[3] = ps.e[0]; pv[4] = ps.e[1];
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) pv[k] = wave_sum(pv[k]);
    // stored now, so that nothing of the pair phase stays live below
    if (lane == 0) {
        glob(cd->f_pair)[ai] = make_double4(pv[0], pv[1], pv[2], 0.0);
        ((gptr<double2>)&glob(cd->e_atom)[ai])[0] = make_double2(0.5 * pv[3], 0.5 * pv[4]);
    }

    double e_cav = 0.0, n_exp = -1.0;
    if (do_cav) {
        // The overlapper's number must fit the low field of acc.
        if (nn >= (1 << ACC_SHIFT)) {
            if (lane == 0) cd->stats->nbr_overflow = 1;
            nn = 0;
        }
        const int nnc = min(nn, MAX_NBR);
        const int N = cd->n_samples;
        const Real drr = (Real)dr;
        // displaced copy of j along e_s covers the sample iff
        //   dot + dr Q_s - c0 - dr^2/(2 R_i) - (dr/R_i) a_s >= 0
        const Real kq = (Real)(dr * dr / (2.0 * roff_i)), k1 = (Real)(dr / roff_i);
        // The shift moves the tested value by drr Q_s - k1 a_s, at most
        // span = drr + k1 max_s |a_s| either way: an exposed sample whose
        // undisplaced value is below -span - guard stays exposed for every
        // axis, a critical one above span + guard stays covered, and their
        // three tests can be skipped with the same decisions.  guard holds
        // the FP32 decision band (mixed) or a rounding pad (FP64).
        const Real guard = MIXED ? (Real)(2.0f * MIXED_BAND) : (Real)1e-9;
        int ncov = 0;
        // net events of the atom itself per axis (the neighbours' reactions go
        // out at once); times the atom's quantum after the wave sum
        int own0 = 0, own1 = 0, own2 = 0;
        if (nn > MAX_NBR) {
            // more neighbours than the LDS list holds: chunks, out of line
            const ChunkArgs ca = {si, off, rbase, nrows, T, nn};
            const ChunkedSasa cs = sasa_chunked<Real>(cd, ca, s_nbr, s_nbr_a, s_ev01, s_ev2);
            ncov = cs.ncov;
            own0 = cs.own[0];
            own1 = cs.own[1];
            own2 = cs.own[2];
        } else {
            // the back part of the list, [MAX_NBR - nback, MAX_NBR), moves
            // down to [nfront, nnc): the list is then contiguous, large caps
            // first.  Each source lies at or above its destination, and a
            // chunk's reads are done before its writes.
            const int nb_back = __builtin_amdgcn_readfirstlane(nback);
            const int nf = __builtin_amdgcn_readfirstlane(nfront);
            for (int c = 0; c < nb_back; c += WAVE) {
                const int v = c + lane;
                // component by component, so that the entry stays in registers
                Real ex = 0, ey = 0, ez = 0, ec = 0;
                int a = 0;
                if (v < nb_back) {
                    const int src = MAX_NBR - nb_back + v;
                    ex = s_nbr[src].ax;
                    ey = s_nbr[src].ay;
                    ez = s_nbr[src].az;
                    ec = s_nbr[src].c0;
                    a = s_nbr_a[src];
                }
                __syncthreads();
                if (v < nb_back) {
                    s_nbr[nf + v].ax = ex;
                    s_nbr[nf + v].ay = ey;
                    s_nbr[nf + v].az = ez;
                    s_nbr[nf + v].c0 = ec;
                    s_nbr_a[nf + v] = a;
                }
                __syncthreads();
            }
            for (int u = lane; u < nnc; u += WAVE) {
                s_ev01[u] = EV_INIT;
                s_ev2[u] = 0;
            }
            __syncthreads();
            const int nlist = __builtin_amdgcn_readfirstlane(nnc);
            for (int kb = 0; kb < N; kb += WAVE * SPL) {
                // step 1: coverage counts of SPL samples per lane
                Real Qx[SPL], Qy[SPL], Qz[SPL], amin[SPL];
                int acc[SPL];
#pragma unroll
                for (int i = 0; i < SPL; ++i) {
                    const int k = kb + lane + WAVE * i;
                    Qx[i] = Qy[i] = Qz[i] = (Real)0;
                    if (k < N) load_q<Real>(cd, k, Qx[i], Qy[i], Qz[i]);
                    acc[i] = 0;
                    amin[i] = (Real)1e30;
                }
                // Blocks of SAT_CHECK neighbours, read once for the four slots.  Once
                // every sample of a slot has two overlappers (decisions
                // outside the FP32 band; a sample with a test inside it is
                // recounted below over the whole list) the rest of the list
                // cannot change its C, and the slot's tests stop; the block
                // loop stops when all four slots have.
                // bit i: slot i holds a sample that can still change (wave-uniform)
                int livem = 0;
#pragma unroll
                for (int i = 0; i < SPL; ++i) {
                    // a lane past N starts saturated, so that it never holds
                    // its slot back (its count is not used)
                    if (kb + lane + WAVE * i >= N) acc[i] = 2 << ACC_SHIFT;
                    if (kb + WAVE * i < N) livem |= 1 << i;
                }
                // one block of SAT_CHECK neighbours from u for the live slots
                auto block = [&](int u) {
                    NbrEntry<Real> e[SAT_CHECK];
#pragma unroll
                    for (int q = 0; q < SAT_CHECK; ++q) e[q] = s_nbr[u + q];
                    int next = 0;
                    const int lm = __builtin_amdgcn_readfirstlane(livem);
                    const int kmul = (1 << ACC_SHIFT) + u - 32;
#pragma unroll
                    for (int i = 0; i < SPL; ++i) {
                        if (!((lm >> i) & 1)) continue;
                        // blk: 32 per covering neighbour plus its index in
                        // the block; its count c = blk >> 5 then adds
                        // c ((1 << ACC_SHIFT) + u) + (blk - 32 c) to acc
                        Real t[SAT_CHECK];
#pragma unroll
                        for (int q = 0; q < SAT_CHECK; ++q) {
                            t[q] = fma(Qz[i], e[q].az, fma(Qy[i], e[q].ay, fma(Qx[i], e[q].ax, -e[q].c0)));
                            if (MIXED) amin[i] = fmin(amin[i], fabs(t[q]));
                        }
                        int blk;
                        if constexpr (MIXED) {
                            static_assert(SAT_CHECK == 4, "four sign bytes per word");
                            blk = block_code(t[0], t[1], t[2], t[3]);
                        } else {
                            blk = 0;
#pragma unroll
                            for (int q = 0; q < SAT_CHECK; ++q) blk += (t[q] >= (Real)0) ? 32 + q : 0;
                        }
                        acc[i] = mad_u24(blk >> 5, kmul, acc[i] + blk);
                        if (__ballot(acc[i] < (2 << ACC_SHIFT))) next |= 1 << i;
                    }
                    livem = next;
                };
                // kept < 0: slot i of lane l holds sample kb + l + WAVE i;
                // else the first `kept` staged samples fill the slots in order
                int kept = -1;
                const bool can_stage = (nnc * (int)sizeof(NbrEntry<Real>) + WAVE * SPL * (int)sizeof(int)) <=
                                       MAX_NBR * (int)sizeof(NbrEntry<Real>);
                int *s_stage = reinterpret_cast<int *>(s_nbr + nnc);
                int u = 0;
                for (; livem && u < COMPACT_AT && u + SAT_CHECK <= nlist; u += SAT_CHECK) block(u);
                if (livem && u == COMPACT_AT && u + SAT_CHECK <= nlist && can_stage) {
                    int pos = 0;
#pragma unroll
                    for (int i = 0; i < SPL; ++i) {
                        const int kl = lane + WAVE * i;
                        const bool valid = kb + kl < N;
                        const bool band = MIXED && amin[i] <= (Real)MIXED_BAND;
                        const bool keep = valid && (acc[i] < (2 << ACC_SHIFT) || band);
                        const unsigned long long m = __ballot(keep);
                        if (keep) s_stage[pos + count_below(m)] = acc[i] | (kl << STAGE_K) | (band ? 1 << 30 : 0);
                        if (valid && !keep) ++ncov;
                        pos += __popcll(m);
                    }
                    kept = __builtin_amdgcn_readfirstlane(pos);
                    __builtin_amdgcn_wave_barrier();
                    int next = 0;
#pragma unroll
                    for (int i = 0; i < SPL; ++i) {
                        int p = lane + WAVE * i;
                        asm volatile("" : "+v"(p));  // recomputed here, not kept (and spilled) from the pass start
                        acc[i] = 2 << ACC_SHIFT;
                        amin[i] = (Real)1e30;
                        Qx[i] = Qy[i] = Qz[i] = (Real)0;
                        if (p < kept) {
                            const int w = s_stage[p];
                            acc[i] = w & ((1 << STAGE_K) - 1);
                            if (w >> 30) amin[i] = (Real)0;
                            load_q<Real>(cd, kb + ((w >> STAGE_K) & 255), Qx[i], Qy[i], Qz[i]);
                        }
                        if (__ballot(acc[i] < (2 << ACC_SHIFT))) next |= 1 << i;
                    }
                    livem = __builtin_amdgcn_readfirstlane(next);
                }
                for (; livem && u + SAT_CHECK <= nlist; u += SAT_CHECK) block(u);
                if (!livem) u = nlist;
                const int lm = __builtin_amdgcn_readfirstlane(livem);
                for (; u < nlist; ++u) {
                    const NbrEntry<Real> e = s_nbr[u];
                    const int inc = (1 << ACC_SHIFT) + u;
#pragma unroll
                    for (int i = 0; i < SPL; ++i) {
                        if (!((lm >> i) & 1)) continue;
                        const Real t = fma(Qz[i], e.az, fma(Qy[i], e.ay, fma(Qx[i], e.ax, -e.c0)));
                        acc[i] += (t >= (Real)0) ? inc : 0;
                        if (MIXED) amin[i] = fmin(amin[i], fabs(t));
                    }
                }
                // sample of lane l in slot i
                auto sample_of = [&](int i, int l) -> int {
                    if (kept < 0) return kb + l + WAVE * i;
                    int p = l + WAVE * i;
                    asm volatile("" : "+v"(p));  // computed at the (rare) use, not kept from the pass start
                    return kb + ((s_stage[p] >> STAGE_K) & 255);
                };
#pragma unroll
                for (int i = 0; i < SPL; ++i) {
                    const bool valid = kept < 0 ? kb + lane + WAVE * i < N : lane + WAVE * i < kept;
                    if (MIXED) {
                        // a test within the band of its threshold: the whole wave
                        // recounts that sample in FP64, one lane per neighbour
                        unsigned long long bm = __ballot(valid && amin[i] <= (Real)MIXED_BAND);
                        while (bm) {
                            const int l = __ffsll((long long)bm) - 1;
                            bm &= bm - 1;
                            const int kl = sample_of(i, l);
                            int part = 0;
                            for (int u = lane; u < nnc; u += WAVE)
                                if (cover_exact(cd, ri, roff_i, kl, s_nbr_a[u], -1)) part += (1 << ACC_SHIFT) + u;
                            part = wave_sum_i(part);
                            if (lane == l) acc[i] = part;
                        }
                    }
                    const int C = acc[i] >> ACC_SHIFT;
                    if (valid && C == 1) {
                        // critically overlapped: only the overlapper's shifted copies can expose it
                        const int k = sample_of(i, lane);
                        const int u = acc[i] & ((1 << ACC_SHIFT) - 1);
                        const NbrEntry<Real> e = s_nbr[u];
                        const int aj = s_nbr_a[u];
                        const Real base = Qx[i] * e.ax + Qy[i] * e.ay + Qz[i] * e.az - e.c0 - kq;
                        const Real span = drr + k1 * fmax(fabs(e.ax), fmax(fabs(e.ay), fabs(e.az)));
                        if (base - span <= guard) {
                            // events: the shifted copies that no longer cover the sample
                            const Real v0 = base + drr * Qx[i] - k1 * e.ax;
                            const Real v1 = base + drr * Qy[i] - k1 * e.ay;
                            const Real v2 = base + drr * Qz[i] - k1 * e.az;
                            int n0 = v0 < (Real)0, n1 = v1 < (Real)0, n2 = v2 < (Real)0;
                            if (MIXED && band3((float)v0, (float)v1, (float)v2)) {
                                n0 += redo((float)v0, cd, ri, roff_i, k, aj, 0);
                                n1 += redo((float)v1, cd, ri, roff_i, k, aj, 1);
                                n2 += redo((float)v2, cd, ri, roff_i, k, aj, 2);
                            }
                            const unsigned inc01 = (unsigned)n0 + ((unsigned)n1 << 16);
                            if (inc01) atomicAdd(&s_ev01[u], inc01);
                            if (n2) atomicAdd(&s_ev2[u], 1);
                        }
                    }
                    if (valid && C >= 1) ++ncov;
                    // step 2 for the exposed samples of this slot: one lane per
                    // neighbour, the samples broadcast from their lanes
                    const unsigned long long em0 = __ballot(valid && C == 0);
                    if (em0) {
#pragma unroll
                        for (int v = 0; v < NSLOT; ++v) {
                            if (WAVE * v >= nnc) break;
                            int u = lane + WAVE * v;
                            // opaque to hoisting: recomputed per pass, not kept (and spilled) across them
                            asm volatile("" : "+v"(u));
                            const bool own = u < nnc;
                            const NbrEntry<Real> e = s_nbr[own ? u : 0];
                            const int aj = s_nbr_a[own ? u : 0];
                            const Real lim = -(drr + k1 * fmax(fabs(e.ax), fmax(fabs(e.ay), fabs(e.az)))) - guard;
                            // the neighbour's constants: base = q . a - (c0 + kq),
                            // copy d tests base + drr q_d - k1 a_d
                            Real cb = e.c0 + kq, sx = k1 * e.ax, sy = k1 * e.ay, sz = k1 * e.az;
                            asm volatile("" : "+v"(sx), "+v"(sy), "+v"(sz));  // kept, not recomputed per sample
                            int d0 = 0, d1 = 0, d2 = 0;
                            unsigned long long em = em0;
                            while (em) {
                                const int l = __ffsll((long long)em) - 1;
                                em &= em - 1;
                                const Real qx = bcast(Qx[i], l), qy = bcast(Qy[i], l), qz = bcast(Qz[i], l);
                                const Real base = fma(qz, e.az, fma(qy, e.ay, qx * e.ax)) - cb;
                                if (own && base >= lim) {
                                    // events: the shifted copies that now cover the sample
                                    const Real v0 = fma(drr, qx, base) - sx;
                                    const Real v1 = fma(drr, qy, base) - sy;
                                    const Real v2 = fma(drr, qz, base) - sz;
                                    d0 -= v0 >= (Real)0;
                                    d1 -= v1 >= (Real)0;
                                    d2 -= v2 >= (Real)0;
                                    if (MIXED && band3((float)v0, (float)v1, (float)v2)) {
                                        const int kx = sample_of(i, l);
                                        d0 += redo((float)v0, cd, ri, roff_i, kx, aj, 0);
                                        d1 += redo((float)v1, cd, ri, roff_i, kx, aj, 1);
                                        d2 += redo((float)v2, cd, ri, roff_i, kx, aj, 2);
                                    }
                                }
                            }
                            // the lane owns neighbour u here, but critical samples of
                            // other lanes add to the same words: keep atomics
                            const unsigned dec01 = (unsigned)d0 + ((unsigned)d1 << 16);
                            if (dec01) atomicAdd(&s_ev01[u], dec01);
                            if (d2) atomicAdd(&s_ev2[u], d2);
                        }
                    }
                }
            }
            __syncthreads();

            // eq F_cav_patch: atom i gains G0_i ev / (N dr) per axis, neighbour j the opposite
            const long long qf = glob(cd->qfix)[ai];
            for (int u = lane; u < nnc; u += WAVE) {
                const unsigned w01 = s_ev01[u];
                const int e0 = (int)(w01 & 0xffffu) - EV_BIAS, e1 = (int)(w01 >> 16) - EV_BIAS, e2 = s_ev2[u];
                if (!(e0 | e1 | e2)) continue;
                const int aj = s_nbr_a[u];
                own0 += e0;
                own1 += e1;
                own2 += e2;
                if (e0) fix_add(&glob(cd->f_cav)[3 * aj + 0], (-(long long)e0 * qf));
                if (e1) fix_add(&glob(cd->f_cav)[3 * aj + 1], (-(long long)e1 * qf));
                if (e2) fix_add(&glob(cd->f_cav)[3 * aj + 2], (-(long long)e2 * qf));
            }
        }
        __syncthreads();
        ncov = wave_sum_i(ncov);
        own0 = wave_sum_i(own0);
        own1 = wave_sum_i(own1);
        own2 = wave_sum_i(own2);
        if (lane == 0) {
            const long long qf = glob(cd->qfix)[ai];
            if (own0) fix_add(&glob(cd->f_cav)[3 * ai + 0], ((long long)own0 * qf));
            if (own1) fix_add(&glob(cd->f_cav)[3 * ai + 1], ((long long)own1 * qf));
            if (own2) fix_add(&glob(cd->f_cav)[3 * ai + 2], ((long long)own2 * qf));
        }
        e_cav = glob(cd->g0)[ai] * (double)(N - ncov) / (double)N;  // eq G_cav_patch
        n_exp = (double)(N - ncov);
    }
    if (lane == 0) ((gptr<double2>)&glob(cd->e_atom)[ai])[1] = make_double2(e_cav, n_exp);
}

// ---------------------------------------------------------------------------
// k_wrench: per-atom wrench (F, r x F) (eqs KCM_01, KCM_02), the suffix sum
// inside each workgroup and the workgroup-local joint torques; the chain
// kernel adds the contribution of later workgroups
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(ATOM_BLOCK) void k_wrench(Batch bt)
{
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    ChainStats *st = cd->stats;
    const int lb = blockIdx.x - bt.blk_off[c];
    if (lb == 0 && threadIdx.x == 0) {
        // end of the iteration: the chain stays active iff it ran, and its
        // forces await the post phase
        const int go = running(st);
        st->active = go;
        if (go) st->pending_post = 1;
    }
    if (!running(st)) return;
    __shared__ double s_w[ATOM_BLOCK / WAVE][WPART];
    const int a = lb * ATOM_BLOCK + threadIdx.x;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = ATOM_BLOCK / WAVE;
    double v[WPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double4 r = make_double4(0, 0, 0, 0);
    if (a < cd->n_atoms) {
        const double inv_fix = 1.0 / FIX_SCALE;
        const double4 fp = cd->f_pair[a];
        const double Fx = fp.x + (double)cd->f_cav[3 * a] * inv_fix;
        const double Fy = fp.y + (double)cd->f_cav[3 * a + 1] * inv_fix;
        const double Fz = fp.z + (double)cd->f_cav[3 * a + 2] * inv_fix;
        r = cd->r[a];
        v[0] = Fx; v[1] = Fy; v[2] = Fz;
        v[3] = r.y * Fz - r.z * Fy; v[4] = r.z * Fx - r.x * Fz; v[5] = r.x * Fy - r.y * Fx;
        const double4 e = cd->e_atom[a];
        v[6] = e.x; v[7] = e.y; v[8] = e.z;
        v[9] = (isfinite(Fx) && isfinite(Fy) && isfinite(Fz)) ? 0.0 : 1.0;
    }
    // inclusive suffix over the workgroup: this atom and every later one
    double S[WPART];
#pragma unroll
    for (int k = 0; k < WPART; ++k) S[k] = v[k];
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
#pragma unroll
        for (int k = 0; k < WPART; ++k) {
            const double y = __shfl_down(S[k], d, WAVE);
            if (lane + d < WAVE) S[k] += y;
        }
    }
    if (lane == 0)
        for (int k = 0; k < WPART; ++k) s_w[w][k] = S[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        double t = 0.0;
        for (int i = w + 1; i < nw; ++i) t += s_w[i][k];
        S[k] += t;
    }
    if (a < cd->n_atoms) {
        const int res = a / APR, slot = a - res * APR;
        if (slot == 4 && cd->n_chi) {
            // side-chain joint of the residue: its whole torque, over HB1..HB3
            // (atoms a+1 .. a+3), about the CA->CB axis through CA
            const double inv_fix = 1.0 / FIX_SCALE;
            const double4 ca = cd->r[a - 2];
            double ux = r.x - ca.x, uy = r.y - ca.y, uz = r.z - ca.z;
            const double inv = 1.0 / sqrt(ux * ux + uy * uy + uz * uz);
            ux *= inv; uy *= inv; uz *= inv;
            double t = 0.0;
            for (int h = 1; h <= 3; ++h) {
                const int b = a + h;
                const double4 fp = cd->f_pair[b], rb = cd->r[b];
                const double Fx = fp.x + (double)cd->f_cav[3 * b] * inv_fix;
                const double Fy = fp.y + (double)cd->f_cav[3 * b + 1] * inv_fix;
                const double Fz = fp.z + (double)cd->f_cav[3 * b + 2] * inv_fix;
                const double dx = rb.x - ca.x, dy = rb.y - ca.y, dz = rb.z - ca.z;
                t += ux * (dy * Fz - dz * Fy) + uy * (dz * Fx - dx * Fz) + uz * (dx * Fy - dy * Fx);
            }
            cd->tau[cd->n_joints + res] = t;
        }
        if (slot == 2 || slot == 8) {
            const int j = 2 * res + (slot == 8 ? 1 : 0);
            const double4 u = cd->jcur[2 * j], p = cd->jcur[2 * j + 1];
            const double mx = S[3] - (p.y * S[2] - p.z * S[1]);
            const double my = S[4] - (p.z * S[0] - p.x * S[2]);
            const double mz = S[5] - (p.x * S[1] - p.y * S[0]);
            cd->tau[j] = u.x * mx + u.y * my + u.z * mz;
        }
    }
    if (threadIdx.x < WPART) {
        double t = 0.0;
        for (int i = 0; i < nw; ++i) t += s_w[i][threadIdx.x];
        cd->wrench_part[WPART * lb + threadIdx.x] = t;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_tau(const Batch &b, hipStream_t s)
{
    if (b.total_jblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tau, dim3(b.total_jblocks), dim3(JOINT_BLOCK), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_stepfk(const Batch &b, int mode, hipStream_t s)
{
    if (b.total_jblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stepfk, dim3(b.total_jblocks), dim3(JOINT_BLOCK), 0, s, b, mode);
    return hipGetLastError();
}

hipError_t launch_gridboot(const Batch &b, hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gridboot, dim3(b.n_chains), dim3(CHAIN_THREADS), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_finish(const Batch &b, hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3((b.n_chains + 255) / 256), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_stats_gather(const Batch &b, ChainStats *out, hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stats_gather, dim3((b.n_chains + 255) / 256), dim3(256), 0, s, b, out);
    return hipGetLastError();
}

hipError_t launch_fold_control(const Batch &b, int mode, double tol, int64_t max_iter, hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_control, dim3((b.n_chains + 255) / 256), dim3(256), 0, s, b, mode, tol, max_iter);
    return hipGetLastError();
}

hipError_t launch_mc_propose(const Batch &b, int mode, const double *delta, const int64_t *delta_off, int trial,
                             hipStream_t s)
{
    if (b.total_jblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mc_propose, dim3(b.total_jblocks), dim3(JOINT_BLOCK), 0, s, b, mode, delta, delta_off,
                       trial);
    return hipGetLastError();
}

hipError_t launch_mc_decide(const Batch &b, int mode, const double *u, int n_trials, int trial, double kT,
                            hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mc_decide, dim3((b.n_chains + 255) / 256), dim3(256), 0, s, b, mode, u, n_trials, trial,
                       kT);
    return hipGetLastError();
}

hipError_t launch_mc_apply(const Batch &b, hipStream_t s)
{
    if (b.total_jblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mc_apply, dim3(b.total_jblocks), dim3(JOINT_BLOCK), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_set_theta(const Batch &b, const double *theta, const int64_t *theta_off, hipStream_t s)
{
    if (b.total_jblocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_theta, dim3(b.total_jblocks), dim3(JOINT_BLOCK), 0, s, b, theta, theta_off);
    return hipGetLastError();
}

hipError_t launch_place(const Batch &b, int mode, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b, mode);
    return hipGetLastError();
}

// Key workgroups (atoms / 256) from which the grid gets a launch of its own:
// the 256-chain batch (3,196) runs faster split, the 1000-residue globule (40)
// with the grid sized in every key workgroup.
constexpr int CELLKEY_SPLIT_BLOCKS = 512;

hipError_t launch_cellkey(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    // the separate sizing launch pays off once the key workgroups are many
    if (b.total_blocks >= CELLKEY_SPLIT_BLOCKS) {
        hipLaunchKernelGGL(k_grid, dim3(b.n_chains), dim3(WAVE), 0, s, b);
        hipLaunchKernelGGL(k_cellkey<false>, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b);
    } else {
        hipLaunchKernelGGL(k_cellkey<true>, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b);
    }
    return hipGetLastError();
}

hipError_t launch_cellscan(const Batch &b, hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    if (b.total_scan_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cellscan, dim3(b.total_scan_blocks), dim3(CHAIN_THREADS), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_scatter(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(b.total_blocks), dim3(ATOM_BLOCK), sizeof(int) * (b.max_scan_chunks + 1), s, b);
    return hipGetLastError();
}

hipError_t launch_rank(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rank, dim3(b.total_blocks), dim3(ATOM_BLOCK), sizeof(int) * (b.max_scan_chunks + 1), s, b);
    return hipGetLastError();
}

hipError_t launch_wrench(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wrench, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b);
    return hipGetLastError();
}

template <int V>
void launch_force_shape(const Batch &b, int precision, hipStream_t s)
{
    constexpr int C = FORCE_SHAPES[V].cpt, S = FORCE_SHAPES[V].satb;
    constexpr bool X = FORCE_SHAPES[V].xcd;
    if (precision == 1)
        hipLaunchKernelGGL((k_force<float, C, S, X>), dim3(b.total_atoms), dim3(WAVE), 0, s, b);
    else
        hipLaunchKernelGGL((k_force<double, C, S, X>), dim3(b.total_atoms), dim3(WAVE), 0, s, b);
}

hipError_t launch_force(const Batch &b, int precision, int shape, hipStream_t s)
{
    if (b.total_atoms <= 0) return hipSuccess;
    static_assert(sizeof(FORCE_SHAPES) / sizeof(FORCE_SHAPES[0]) == FORCE_SHAPE_COUNT, "shape table");
    switch (shape) {
    case 1: launch_force_shape<1>(b, precision, s); break;
    case 2: launch_force_shape<2>(b, precision, s); break;
    case 3: launch_force_shape<3>(b, precision, s); break;
    default: launch_force_shape<0>(b, precision, s); break;
    }
    return hipGetLastError();
}

}  // namespace kcm
