// kcm_kernels.hip -- gfx950 kernels of one KCM iteration.
//
//   k_chain     one workgroup per chain.  Post phase of the previous
//               iteration: link wrenches and the suffix (row) scan of eq 04_9
//               giving tau_k = u_k . (T_k - p_k x F_k) (eqs KCM_01-KCM_06),
//               then the compliance step (eq KCM_07).  Then forward
//               kinematics of the new angles as an ordered prefix scan of
//               rigid transforms (eqs kin_02-kin_04, r1; prefix computation
//               item 1 of Sec. 3.5) and the cell grid of Sec. 3.2, sized from
//               the previous bounding box plus a margin (atoms outside it are
//               clamped to the border cells, which keeps every neighbour
//               within the stencil).
//   k_place     one thread per atom: r_a = G_link(a) r0_a, cell key, cell
//               count, bounding box of the new positions.
//   k_cellscan  one workgroup per chain: cell starts by an exclusive scan.
//   k_scatter   one thread per atom: counting-sort scatter by cell key.
//   k_rank      one thread per atom: stable slot inside the cell, gather.
//   k_cellsort  one thread per cell: restores atom order inside the cell
//               (the sort is then stable, so everything downstream is
//               deterministic) and gathers positions/parameters in cell order.
//   k_force     one workgroup per atom, atoms in cell order: stencil
//               candidates in FP64, Coulomb + LJ (eqs 02-03_9) over the full
//               pair list, solvation neighbours in LDS, and the SASA
//               enumeration of Algorithm 1 with the C-state rules (Sec. 3.4):
//               coverage counts with one sample per lane, then the displaced
//               tests for the compacted exposed samples only.  Solvation
//               events are scattered as fixed-point integers, so every sum is
//               order independent.
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

// Joint j: right-hand rotation by (theta_j - pi) about the zero-position axis
// line through p0_j with direction u0_j.
__device__ __forceinline__ Xf joint_xf(const double4 *__restrict__ joint0, const double *__restrict__ theta, int j)
{
    const double4 u = joint0[2 * j], p = joint0[2 * j + 1];
    double s, c;
    sincos(theta[j] - PI_D, &s, &c);
    const double k = 1.0 - c;
    Xf x;
    x.r[0] = c + u.x * u.x * k;       x.r[1] = u.x * u.y * k - u.z * s; x.r[2] = u.x * u.z * k + u.y * s;
    x.r[3] = u.y * u.x * k + u.z * s; x.r[4] = c + u.y * u.y * k;       x.r[5] = u.y * u.z * k - u.x * s;
    x.r[6] = u.z * u.x * k - u.y * s; x.r[7] = u.z * u.y * k + u.x * s; x.r[8] = c + u.z * u.z * k;
#pragma unroll
    for (int i = 0; i < 3; ++i) x.t[i] = ((&p.x)[i]) - (x.r[3 * i] * p.x + x.r[3 * i + 1] * p.y + x.r[3 * i + 2] * p.z);
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

__device__ __forceinline__ double4 place_atom(const ChainDev *cd, int a)
{
    const double *L = cd->xform + 12 * link_of_atom(a);
    const double4 q = cd->r0[a];
    double4 r;
    r.x = L[0] * q.x + L[1] * q.y + L[2] * q.z + L[9];
    r.y = L[3] * q.x + L[4] * q.y + L[5] * q.z + L[10];
    r.z = L[6] * q.x + L[7] * q.y + L[8] * q.z + L[11];
    r.w = 0.0;
    return r;
}

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

constexpr double GRID_MARGIN = 2.0;  // A added around the previous bounding box

// ---------------------------------------------------------------------------
// k_chain: post phase of the previous iteration, then kinematics and grid
// ---------------------------------------------------------------------------
constexpr int FK_REG = 2;  // joints per thread kept in registers (J <= FK_REG * blockDim)

// Post phase of the previous iteration for this thread's joints [j0, j1).
// th[] holds their angles on entry (when the chunk fits FK_REG) and the
// updated angles on exit.
__device__ void post_phase(const ChainDev *cd, int j0, int j1, double (&th)[FK_REG], bool in_reg, int *s_flag,
                           double *s_red, double (*s_w)[6])
{
    ChainStats *st = cd->stats;
    const int n = cd->n_atoms;
    const int nblk = (n + ATOM_BLOCK - 1) / ATOM_BLOCK;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (WAVE - 1), w = tid / WAVE, nw = nt / WAVE;
    double *__restrict__ part = cd->wrench_part;
    double *__restrict__ tau = cd->tau;
    double *__restrict__ theta = cd->theta;
    double *__restrict__ dtheta = cd->dtheta;
    const uint8_t *__restrict__ mask = cd->mask;
    const double4 *__restrict__ jcur = cd->jcur;

    // energies and the failure flag: plain sums of the per-workgroup partials
    double E[4] = {0, 0, 0, 0};
    for (int b = tid; b < nblk; b += nt) {
        E[0] += part[WPART * b + 6];
        E[1] += part[WPART * b + 7];
        E[2] += part[WPART * b + 8];
        E[3] += part[WPART * b + 9];
    }
    block_sum<4>(E, s_red);

    // exclusive suffix over workgroups, in place: part[b][0..5] becomes the
    // wrench of every atom after workgroup b (processed from the last chunk)
    double carry[6] = {0, 0, 0, 0, 0, 0};
    for (int c0 = ((nblk - 1) / nt) * nt; c0 >= 0; c0 -= nt) {
        const int b = c0 + tid;
        double v[6], S[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = (b < nblk) ? part[WPART * b + k] : 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) S[k] = v[k];
#pragma unroll
        for (int d = 1; d < WAVE; d <<= 1) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const double y = __shfl_down(S[k], d, WAVE);
                if (lane + d < WAVE) S[k] += y;
            }
        }
        if (lane == 0)
            for (int k = 0; k < 6; ++k) s_w[w][k] = S[k];
        __syncthreads();
        double later[6], tot[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double t = 0.0, u = 0.0;
            for (int i = 0; i < nw; ++i) {
                u += s_w[i][k];
                if (i > w) t += s_w[i][k];
            }
            later[k] = t;
            tot[k] = u;
        }
        if (b < nblk)
            for (int k = 0; k < 6; ++k) part[WPART * b + k] = carry[k] + later[k] + (S[k] - v[k]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 6; ++k) carry[k] += tot[k];
    }

    // tau_j = (workgroup-local part from k_wrench) + u_j . (T_later - p_j x F_later)
    double tmax = 0.0;
    bool tbad = false;
    for (int j = j0; j < j1; ++j) {
        const int first = APR * (j >> 1) + ((j & 1) ? 8 : 2);  // first atom of link j+1
        const double *S = part + WPART * (first / ATOM_BLOCK);
        const double4 u = jcur[2 * j], p = jcur[2 * j + 1];
        const double mx = S[3] - (p.y * S[2] - p.z * S[1]);
        const double my = S[4] - (p.z * S[0] - p.x * S[2]);
        const double mz = S[5] - (p.x * S[1] - p.y * S[0]);
        const double t = tau[j] + (u.x * mx + u.y * my + u.z * mz);
        tau[j] = t;
        if (!isfinite(t)) tbad = true;
        if (mask[j]) tmax = fmax(tmax, fabs(t));
    }
    tmax = block_max(tmax, s_red);
    const double anybad = block_max(tbad ? 1.0 : 0.0, s_red);
    if (E[3] > 0.0 || anybad > 0.0) {
        if (tid == 0) {
            st->e_elec = E[0]; st->e_vdw = E[1]; st->e_cav = E[2];
            st->status = -4;
            st->active = 0;
            *s_flag = 0;
        }
        __syncthreads();
        return;
    }
    const double kappa = cd->kappa, s = cd->max_step;
    double scale;
    if (cd->step_rule == 1) scale = tmax > 0.0 ? s / tmax : 0.0;
    else if (cd->step_rule == 2) scale = kappa;
    else scale = (kappa * tmax > s) ? s / tmax : kappa;
    double mxd = 0.0;
#pragma unroll
    for (int i = 0; i < FK_REG; ++i) {
        const int j = j0 + i;
        if (!in_reg || j >= j1) continue;
        const double d = mask[j] ? scale * tau[j] : 0.0;
        dtheta[j] = d;
        mxd = fmax(mxd, fabs(d));
        double t = th[i] + d;
        if (t > PI_D) t -= 2.0 * PI_D;
        if (t <= -PI_D) t += 2.0 * PI_D;
        th[i] = t;
        theta[j] = t;
    }
    if (!in_reg) {
        for (int j = j0; j < j1; ++j) {
            const double d = mask[j] ? scale * tau[j] : 0.0;
            dtheta[j] = d;
            mxd = fmax(mxd, fabs(d));
            double t = theta[j] + d;
            if (t > PI_D) t -= 2.0 * PI_D;
            if (t <= -PI_D) t += 2.0 * PI_D;
            theta[j] = t;
        }
    }
    mxd = block_max(mxd, s_red);
    if (tid == 0) {
        st->e_elec = E[0]; st->e_vdw = E[1]; st->e_cav = E[2];
        st->max_tau = tmax;
        st->max_dtheta = mxd;
        st->iterations += 1;
        if (st->nbr_overflow) st->status = -6;
        if (st->tol > 0.0 && mxd < st->tol) {
            st->converged = 1;
            st->active = 0;
        }
        if (st->iterations >= st->iter_limit) st->active = 0;
        *s_flag = st->active;
    }
    __syncthreads();
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

// Ordered scan G_j = T_0 o T_1 o ... o T_j over the block for this thread's
// joints [j0, j1); th[] holds their angles when in_reg.  s_x: [16][12].
__device__ void fk_phase(const ChainDev *cd, int j0, int j1, const double (&th)[FK_REG], bool in_reg, double (*s_x)[12])
{
    const double4 *__restrict__ joint0 = cd->joint0;
    const double *__restrict__ theta = cd->theta;
    double *__restrict__ xform = cd->xform;
    double4 *__restrict__ jcur = cd->jcur;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (WAVE - 1), w = tid / WAVE, nw = nt / WAVE;
    Xf x = xf_identity();
    if (in_reg) {
#pragma unroll
        for (int i = 0; i < FK_REG; ++i)
            if (j0 + i < j1) x = xf_mul(x, joint_xf_of(joint0[2 * (j0 + i)], joint0[2 * (j0 + i) + 1], th[i]));
    } else {
        for (int j = j0; j < j1; ++j) x = xf_mul(x, joint_xf(joint0, theta, j));
    }
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        Xf y = xf_shfl_up(x, d);
        if (lane >= d) x = xf_mul(y, x);
    }
    if (lane == WAVE - 1) xf_store(s_x[w], x);
    __syncthreads();
    if (w == 0) {
        // ordered scan of the wave totals inside wave 0
        Xf v = lane < nw ? xf_load(s_x[lane]) : xf_identity();
#pragma unroll
        for (int d = 1; d < CHAIN_THREADS / WAVE; d <<= 1) {
            Xf y = xf_shfl_up(v, d);
            if (lane >= d) v = xf_mul(y, v);
        }
        Xf e = xf_shfl_up(v, 1);
        if (lane == 0) e = xf_identity();
        if (lane < nw) xf_store(s_x[lane], e);
    }
    __syncthreads();
    Xf ex = xf_shfl_up(x, 1);
    if (lane == 0) ex = xf_identity();
    Xf G = xf_mul(xf_load(s_x[w]), ex);
    if (in_reg) {
#pragma unroll
        for (int i = 0; i < FK_REG; ++i)
            if (j0 + i < j1) {
                G = xf_mul(G, joint_xf_of(joint0[2 * (j0 + i)], joint0[2 * (j0 + i) + 1], th[i]));
                fk_emit(G, j0 + i, joint0, xform, jcur);
            }
    } else {
        for (int j = j0; j < j1; ++j) {
            G = xf_mul(G, joint_xf(joint0, theta, j));
            fk_emit(G, j, joint0, xform, jcur);
        }
    }
    if (tid == 0) xf_store(xform, xf_identity());
    __syncthreads();
}

__global__ __launch_bounds__(CHAIN_THREADS) void k_chain(Batch bt, int do_post, int do_fk)
{
    const ChainDev *cd = bt.table[blockIdx.x];
    ChainStats *st = cd->stats;
    if (!st->active) return;
    __shared__ double s_x[CHAIN_THREADS / WAVE][12];
    __shared__ double s_w[CHAIN_THREADS / WAVE][6];
    __shared__ double s_red[CHAIN_THREADS / WAVE * 6];
    __shared__ int s_flag;
    __shared__ double s_bb[6];
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & (WAVE - 1), w = tid / WAVE, nw = nt / WAVE;
    if (tid == 0) s_flag = 1;
    const int J = cd->n_joints;
    const int chunk = (J + nt - 1) / nt;
    const int j0 = min(J, tid * chunk), j1 = min(J, j0 + chunk);
    const bool in_reg = chunk <= FK_REG;
    double th[FK_REG];
#pragma unroll
    for (int i = 0; i < FK_REG; ++i) th[i] = (in_reg && j0 + i < j1) ? cd->theta[j0 + i] : 0.0;
    __syncthreads();
    if (do_post && st->pending_post) {
        post_phase(cd, j0, j1, th, in_reg, &s_flag, s_red, s_w);
        if (tid == 0) st->pending_post = 0;
    }
    if (!do_fk || !s_flag) return;
    fk_phase(cd, j0, j1, th, in_reg, s_x);

    // bounding box that sizes this iteration's grid
    const int n = cd->n_atoms;
    if (st->need_grid) {
        double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
        bool finite = true;
        for (int a = tid; a < n; a += nt) {
            const double4 r = place_atom(cd, a);
            finite = finite && isfinite(r.x) && isfinite(r.y) && isfinite(r.z);
            lo[0] = fmin(lo[0], r.x); lo[1] = fmin(lo[1], r.y); lo[2] = fmin(lo[2], r.z);
            hi[0] = fmax(hi[0], r.x); hi[1] = fmax(hi[1], r.y); hi[2] = fmax(hi[2], r.z);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
        const int bad_w = __any(!finite);
        if (lane == 0) {
            for (int k = 0; k < 3; ++k) { s_red[w * 6 + k] = lo[k]; s_red[w * 6 + 3 + k] = hi[k]; }
            if (bad_w) s_flag = 0;
        }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < 3; ++k) { s_bb[k] = DBL_MAX; s_bb[3 + k] = -DBL_MAX; }
            for (int i = 0; i < nw; ++i)
                for (int k = 0; k < 3; ++k) {
                    s_bb[k] = fmin(s_bb[k], s_red[i * 6 + k]);
                    s_bb[3 + k] = fmax(s_bb[3 + k], s_red[i * 6 + 3 + k]);
                }
            if (!s_flag) s_bb[0] = NAN;
            st->need_grid = 0;
        }
    } else {
        const int nblk = (n + ATOM_BLOCK - 1) / ATOM_BLOCK;
        double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
        for (int b = tid; b < nblk; b += nt)
            for (int k = 0; k < 3; ++k) {
                lo[k] = fmin(lo[k], cd->bbox_part[6 * b + k]);
                hi[k] = fmax(hi[k], cd->bbox_part[6 * b + 3 + k]);
            }
#pragma unroll
        for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
        if (lane == 0)
            for (int k = 0; k < 3; ++k) { s_red[w * 6 + k] = lo[k]; s_red[w * 6 + 3 + k] = hi[k]; }
        __syncthreads();
        if (tid == 0) {
            for (int k = 0; k < 3; ++k) { s_bb[k] = DBL_MAX; s_bb[3 + k] = -DBL_MAX; }
            for (int i = 0; i < nw; ++i)
                for (int k = 0; k < 3; ++k) {
                    s_bb[k] = fmin(s_bb[k], s_red[i * 6 + k]);
                    s_bb[3 + k] = fmax(s_bb[3 + k], s_red[i * 6 + 3 + k]);
                }
        }
    }
    __syncthreads();

    if (tid == 0) {
        const double reach_len = fmax(cd->cutoff, 2.0 * cd->roff_max + cd->delta_r) + 1e-7;
        double L3[3], H3[3];
        bool ok = true;
        for (int k = 0; k < 3; ++k) {
            L3[k] = s_bb[k] - GRID_MARGIN;
            H3[k] = s_bb[3 + k] + GRID_MARGIN;
            ok = ok && isfinite(L3[k]) && isfinite(H3[k]) && H3[k] >= L3[k] && (H3[k] - L3[k]) < 1e7;
        }
        double cell = fmax(cd->cell_min, reach_len / MAX_REACH);
        long long dims[3] = {1, 1, 1};
        for (int it = 0; ok && it < 200; ++it) {
            for (int k = 0; k < 3; ++k) dims[k] = (long long)floor((H3[k] - L3[k]) / cell) + 1;
            if (dims[0] * dims[1] * dims[2] <= cd->cap_cells) break;
            cell *= 1.2599210498948732;
        }
        ok = ok && dims[0] * dims[1] * dims[2] <= cd->cap_cells;
        Grid g;
        for (int k = 0; k < 3; ++k) { g.origin[k] = ok ? L3[k] : 0.0; g.dims[k] = ok ? (int)dims[k] : 1; }
        g.cell = cell;
        g.inv_cell = 1.0 / cell;
        g.reach = max(1, (int)ceil(reach_len / cell - 1e-9));
        g.n_cells = ok ? (int)(dims[0] * dims[1] * dims[2]) : 0;
        g.pad = 0;
        *cd->grid = g;
        s_flag = ok ? g.n_cells : 0;
        if (!ok) {
            st->status = -4;
            st->active = 0;
        }
    }
    __syncthreads();
    const int nc = s_flag;
    for (int c = tid; c < nc; c += nt) cd->cell_count[c] = 0;
}

// ---------------------------------------------------------------------------
// k_place: positions, cell keys, cell counts, bounding box
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(ATOM_BLOCK) void k_place(Batch bt)
{
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    if (!cd->stats->active) return;
    const int a = (blockIdx.x - bt.blk_off[c]) * ATOM_BLOCK + threadIdx.x;
    const int n = cd->n_atoms;
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    if (a < n) {
        const Grid g = *cd->grid;
        const double4 r = place_atom(cd, a);
        cd->r[a] = r;
        const int key = cell_of(g, r);
        cd->cell_key[a] = key;
        atomicAdd(&cd->cell_count[key], 1);
        cd->f_cav[3 * a] = 0;
        cd->f_cav[3 * a + 1] = 0;
        cd->f_cav[3 * a + 2] = 0;
        lo[0] = r.x; lo[1] = r.y; lo[2] = r.z;
        hi[0] = r.x; hi[1] = r.y; hi[2] = r.z;
    }
    __shared__ double s_bb[ATOM_BLOCK / WAVE][6];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
    for (int k = 0; k < 3; ++k) { lo[k] = wave_min(lo[k]); hi[k] = wave_max(hi[k]); }
    if (lane == 0)
        for (int k = 0; k < 3; ++k) { s_bb[w][k] = lo[k]; s_bb[w][3 + k] = hi[k]; }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double v = s_bb[0][k];
        for (int i = 1; i < ATOM_BLOCK / WAVE; ++i) v = (k < 3) ? fmin(v, s_bb[i][k]) : fmax(v, s_bb[i][k]);
        cd->bbox_part[6 * (blockIdx.x - bt.blk_off[c]) + k] = v;
    }
}

// ---------------------------------------------------------------------------
// k_cellscan: cell_start = exclusive scan of the counts (LDS chunks, carry)
// ---------------------------------------------------------------------------
constexpr int SCAN_CHUNK = 16384;

__global__ __launch_bounds__(CHAIN_THREADS) void k_cellscan(Batch bt)
{
    const ChainDev *cd = bt.table[blockIdx.x];
    if (!cd->stats->active) return;
    __shared__ int s_cnt[SCAN_CHUNK];
    __shared__ int s_int[CHAIN_THREADS / WAVE];
    const int nc = cd->grid->n_cells;
    const int *__restrict__ count = cd->cell_count;
    int *__restrict__ start = cd->cell_start;
    int *__restrict__ cursor = cd->cell_cursor;
    const int tid = threadIdx.x, nt = blockDim.x;
    constexpr int PER = SCAN_CHUNK / CHAIN_THREADS;
    int carry = 0;
    for (int c0 = 0; c0 < nc; c0 += SCAN_CHUNK) {
        const int m = min(SCAN_CHUNK, nc - c0);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = k * nt + tid;
            s_cnt[i] = i < m ? count[c0 + i] : 0;
        }
        __syncthreads();
        int loc = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) loc += s_cnt[tid * PER + k];
        int total = 0;
        int run = carry + block_excl_scan(loc, s_int, &total);
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int v = s_cnt[tid * PER + k];
            s_cnt[tid * PER + k] = run;
            run += v;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = k * nt + tid;
            if (i < m) {
                start[c0 + i] = s_cnt[i];
                cursor[c0 + i] = 0;
            }
        }
        carry += total;
        __syncthreads();
    }
    if (tid == 0) start[nc] = carry;
}

// ---------------------------------------------------------------------------
// k_scatter: counting-sort scatter by cell key (slot order inside a cell left
// to the atomics), then k_rank: each atom takes as its slot the number of
// atoms of its cell with a smaller index, so the final cell order is stable
// and everything downstream is deterministic; it gathers positions and
// parameters into that order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(ATOM_BLOCK) void k_scatter(Batch bt)
{
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    const ChainDev *cd = bt.table[c];
    if (!cd->stats->active) return;
    const int a = (blockIdx.x - bt.blk_off[c]) * ATOM_BLOCK + threadIdx.x;
    if (a >= cd->n_atoms) return;
    const int key = cd->cell_key[a];
    cd->s_tmp[cd->cell_start[key] + atomicAdd(&cd->cell_cursor[key], 1)] = a;
}

__global__ __launch_bounds__(ATOM_BLOCK) void k_rank(Batch bt)
{
    const int c = find_block_owner(bt.blk_off, bt.n_chains, blockIdx.x);
    const ChainDev *cd = bt.table[c];
    if (!cd->stats->active) return;
    const int a = (blockIdx.x - bt.blk_off[c]) * ATOM_BLOCK + threadIdx.x;
    if (a >= cd->n_atoms) return;
    const int key = cd->cell_key[a];
    const double4 r = cd->r[a];
    const double4 p = cd->aparam[a];
    const int b = cd->cell_start[key], e = cd->cell_start[key + 1];
    const int *__restrict__ tmp = cd->s_tmp;
    int rank = 0;
    for (int s = b; s < e; ++s) rank += tmp[s] < a ? 1 : 0;
    const int pos = b + rank;
    cd->s_idx[pos] = a;
    cd->s_cell[pos] = key;
    cd->s_r[pos] = r;
    cd->s_p[pos] = p;
}

// ---------------------------------------------------------------------------
// k_force: Coulomb + LJ + SASA enumeration, one workgroup per atom
// ---------------------------------------------------------------------------
// A solvation neighbour j of atom i: offset a = r_j - r_i and the threshold c0 =
// (R_i^2 + |a|^2 - R_j^2) / (2 R_i): sample q_k = r_i + R_i Q_k is covered by j iff
// Q_k . a >= c0 (the same test as ||q_k - r_j|| <= R_j).
template <typename Real>
struct NbrEntry {
    Real ax, ay, az, c0;
};

// FP64 decision in absolute coordinates: is sample k of atom i covered by the
// offset sphere of sorted atom sj, shifted by delta_r along axis s (s < 0: not
// shifted)?
__device__ __forceinline__ bool cover_exact(const ChainDev *cd, const double4 &ri, double roff_i, int k, int sj, int s)
{
    const double4 q = cd->q64[k];
    const double qx = ri.x + roff_i * q.x, qy = ri.y + roff_i * q.y, qz = ri.z + roff_i * q.z;
    double4 c = cd->s_r[sj];
    if (s == 0) c.x += cd->delta_r;
    if (s == 1) c.y += cd->delta_r;
    if (s == 2) c.z += cd->delta_r;
    const double rj = cd->s_p[sj].w;
    const double dx = qx - c.x, dy = qy - c.y, dz = qz - c.z;
    return dx * dx + dy * dy + dz * dz - rj * rj <= 0.0;
}

template <typename Real, bool MIXED>
__device__ __forceinline__ bool test_cover(Real v, Real thr, const ChainDev *cd, const double4 &ri, double roff_i, int k,
                                           int sj, int s)
{
    bool hit = v >= thr;
    if (MIXED) {
        if (fabsf((float)(v - thr)) <= MIXED_BAND) hit = cover_exact(cd, ri, roff_i, k, sj, s);
    }
    return hit;
}

template <typename Real>
__device__ __forceinline__ void load_q(const ChainDev *cd, int k, Real &x, Real &y, Real &z)
{
    if (sizeof(Real) == 4) {
        const float4 q = cd->q32[k];
        x = (Real)q.x; y = (Real)q.y; z = (Real)q.z;
    } else {
        const double4 q = cd->q64[k];
        x = (Real)q.x; y = (Real)q.y; z = (Real)q.z;
    }
}

template <typename Real>
__global__ __launch_bounds__(FORCE_THREADS) void k_force(Batch bt)
{
    constexpr bool MIXED = sizeof(Real) == 4;
    constexpr int MAX_ROWS = (2 * MAX_REACH + 1) * (2 * MAX_REACH + 1);
    __shared__ NbrEntry<Real> s_nbr[MAX_NBR];
    __shared__ int s_nbr_j[MAX_NBR];
    __shared__ int s_ev[MAX_NBR * 3];
    __shared__ int s_row_beg[MAX_ROWS];
    __shared__ int s_row_off[MAX_ROWS + 1];
    __shared__ int s_exp[FORCE_THREADS];
    __shared__ double s_red[(FORCE_THREADS / WAVE) * 5];
    __shared__ int s_nn, s_ncov, s_nexp;
    __shared__ unsigned long long s_own[3];

    const int c = find_block_owner(bt.atom_off, bt.n_chains, blockIdx.x);
    ChainDev *cd = bt.table[c];
    if (!cd->stats->active) return;
    const int si = blockIdx.x - bt.atom_off[c];
    const int tid = threadIdx.x, nt = blockDim.x;

    const Grid g = *cd->grid;
    const double4 ri = cd->s_r[si];
    const double4 pi = cd->s_p[si];
    const int ai = cd->s_idx[si];
    const int key = cd->s_cell[si];
    const int dxn = g.dims[0], dyn = g.dims[1], dzn = g.dims[2];
    const int cx = key % dxn, cy = (key / dxn) % dyn, cz = key / (dxn * dyn);
    const int R = g.reach, side = 2 * R + 1, nrows = side * side;

    // stencil rows: for each (dy, dz) one contiguous run of cells along x
    for (int t = tid; t < nrows; t += nt) {
        const int y = cy + (t % side) - R, z = cz + (t / side) - R;
        int beg = 0, cnt = 0;
        if (y >= 0 && y < dyn && z >= 0 && z < dzn) {
            const int xl = max(0, cx - R), xh = min(dxn - 1, cx + R);
            const int base = (z * dyn + y) * dxn;
            beg = cd->cell_start[base + xl];
            cnt = cd->cell_start[base + xh + 1] - beg;
        }
        s_row_beg[t] = beg;
        s_row_off[t] = cnt;
    }
    for (int t = tid; t < 3 * MAX_NBR; t += nt) s_ev[t] = 0;
    if (tid == 0) {
        s_nn = 0;
        s_ncov = 0;
        s_nexp = 0;
        s_own[0] = s_own[1] = s_own[2] = 0ull;
    }
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int t = 0; t < nrows; ++t) {
            const int cnt = s_row_off[t];
            s_row_off[t] = run;
            run += cnt;
        }
        s_row_off[nrows] = run;
    }
    __syncthreads();
    const int T = s_row_off[nrows];

    const int terms = cd->terms;
    const bool do_elec = terms & 1, do_vdw = terms & 2, do_cav = terms & 4;
    const bool do_pair = do_elec || do_vdw;
    const double cut2 = cd->cutoff * cd->cutoff;
    const double roff_i = pi.w;
    const double dr = cd->delta_r;
    const int res_i = ai / APR, slot_i = ai - res_i * APR;
    const uint32_t m12 = cd->m12[slot_i], m13 = cd->m13[slot_i], m14 = cd->m14[slot_i];
    const Real w13 = (Real)cd->w13, w14e = (Real)cd->w14e, w14v = (Real)cd->w14v;
    const Real coul = (Real)cd->coulomb;
    const Real qi = (Real)pi.x, Ri = (Real)pi.y, sei = (Real)pi.z;

    Real fx = 0, fy = 0, fz = 0;
    double ee = 0.0, evw = 0.0;
    for (int k = tid; k < T; k += nt) {
        int rlo = 0, rhi = nrows;
        while (rhi - rlo > 1) {
            const int mid = (rlo + rhi) >> 1;
            if (s_row_off[mid] <= k) rlo = mid; else rhi = mid;
        }
        const int sj = s_row_beg[rlo] + (k - s_row_off[rlo]);
        if (sj == si) continue;
        const double4 rj = cd->s_r[sj];
        const double ddx = rj.x - ri.x, ddy = rj.y - ri.y, ddz = rj.z - ri.z;
        const double d2 = ddx * ddx + ddy * ddy + ddz * ddz;
        const bool in_pair = do_pair && d2 <= cut2;
        bool in_cav = false;
        double4 pj;
        if (in_pair || do_cav) pj = cd->s_p[sj];
        if (do_cav) {
            const double lim = roff_i + pj.w + dr;
            in_cav = d2 <= lim * lim;
        }
        if (in_pair) {
            const int aj = cd->s_idx[sj];
            const int res_j = aj / APR, dres = res_j - res_i;
            Real we = do_elec ? (Real)1 : (Real)0, wv = do_vdw ? (Real)1 : (Real)0;
            if (dres >= -1 && dres <= 1) {
                const uint32_t bit = 1u << ((dres + 1) * APR + (aj - res_j * APR));
                if (m12 & bit) { we = 0; wv = 0; }
                else if (m13 & bit) { we *= w13; wv *= w13; }
                else if (m14 & bit) { we *= w14e; wv *= w14v; }
            }
            if (we != (Real)0 || wv != (Real)0) {
                const Real rx = (Real)ddx, ry = (Real)ddy, rz = (Real)ddz;
                const Real inv2 = (Real)1 / (Real)d2;
                // eq 02 with eps = k_d d: E = (C/k_d) q_i q_j / d^2
                const Real eel = we * coul * qi * (Real)pj.x * inv2;
                // eq 03: E = eps_ij [(D/d)^12 - 2 (D/d)^6], D = R_i + R_j, eps_ij = sqrt(eps_i eps_j)
                const Real D = Ri + (Real)pj.y;
                const Real s2 = D * D * inv2, s6 = s2 * s2 * s2, s12 = s6 * s6;
                const Real eij = sei * (Real)pj.z;
                const Real elj = wv * eij * (s12 - (Real)2 * s6);
                // |F|/d along r_i - r_j: 2 E_elec/d^2 + 12 eps (s12 - s6)/d^2
                const Real fsc = ((Real)2 * eel + (Real)12 * wv * eij * (s12 - s6)) * inv2;
                fx -= fsc * rx;
                fy -= fsc * ry;
                fz -= fsc * rz;
                ee += (double)eel;
                evw += (double)elj;
            }
        }
        if (in_cav) {
            const int slot = atomicAdd(&s_nn, 1);
            if (slot < MAX_NBR) {
                const double Rj = pj.w;
                NbrEntry<Real> e;
                e.ax = (Real)ddx; e.ay = (Real)ddy; e.az = (Real)ddz;
                e.c0 = (Real)((roff_i * roff_i + d2 - Rj * Rj) / (2.0 * roff_i));
                s_nbr[slot] = e;
                s_nbr_j[slot] = sj;
            }
        }
    }

    // pair force and energy of atom i (each unordered pair is seen from both ends)
    double pv[5] = {(double)fx, (double)fy, (double)fz, ee, evw};
    block_sum<5>(pv, s_red);

    double e_cav = 0.0, n_exp = -1.0;
    if (do_cav) {
        const int nn_all = s_nn;
        const int nn = min(nn_all, MAX_NBR);
        if (nn_all > MAX_NBR && tid == 0) cd->stats->nbr_overflow = 1;
        const int N = cd->n_samples;
        const Real drr = (Real)dr;
        // displaced copy of j along e_s covers the sample iff
        //   dot + dr Q_s >= c0 + dr^2/(2 R_i) + (dr/R_i) a_s
        const Real kq = (Real)(dr * dr / (2.0 * roff_i)), k1 = (Real)(dr / roff_i);
        int ncov = 0;
        for (int kb = 0; kb < N; kb += nt) {
            if (kb > 0) {
                if (tid == 0) s_nexp = 0;
                __syncthreads();
            }
            const int k = kb + tid;
            if (k < N) {
                Real Qx, Qy, Qz;
                load_q<Real>(cd, k, Qx, Qy, Qz);
                // step 1: acc = 65536 * (covering neighbours) + (sum of their slots), so
                // acc >> 16 == 1 leaves the single overlapper in the low bits
                int acc = 0;
                Real amin = (Real)1e30;
                for (int u = 0; u < nn; ++u) {
                    const NbrEntry<Real> e = s_nbr[u];
                    const Real t = fma(Qz, e.az, fma(Qy, e.ay, fma(Qx, e.ax, -e.c0)));
                    acc += (t >= (Real)0) ? (65536 + u) : 0;
                    if (MIXED) amin = fmin(amin, fabs(t));
                }
                if (MIXED && amin <= (Real)MIXED_BAND) {
                    acc = 0;
                    for (int u = 0; u < nn; ++u)
                        if (cover_exact(cd, ri, roff_i, k, s_nbr_j[u], -1)) acc += 65536 + u;
                }
                const int C = acc >> 16;
                if (C == 0) {
                    s_exp[atomicAdd(&s_nexp, 1)] = k;
                } else if (C == 1) {
                    // critically overlapped: only the overlapper's shifted copies can expose it
                    const int u = acc & 0xFFFF;
                    const NbrEntry<Real> e = s_nbr[u];
                    const Real base = Qx * e.ax + Qy * e.ay + Qz * e.az - e.c0 - kq;
                    if (!test_cover<Real, MIXED>(base + drr * Qx - k1 * e.ax, (Real)0, cd, ri, roff_i, k, s_nbr_j[u], 0)) atomicAdd(&s_ev[3 * u + 0], 1);
                    if (!test_cover<Real, MIXED>(base + drr * Qy - k1 * e.ay, (Real)0, cd, ri, roff_i, k, s_nbr_j[u], 1)) atomicAdd(&s_ev[3 * u + 1], 1);
                    if (!test_cover<Real, MIXED>(base + drr * Qz - k1 * e.az, (Real)0, cd, ri, roff_i, k, s_nbr_j[u], 2)) atomicAdd(&s_ev[3 * u + 2], 1);
                }
                if (C >= 1) ++ncov;
            }
            __syncthreads();
            // step 2 for the exposed samples of this batch: every (sample, neighbour) pair
            const int nexp = s_nexp;
            const int work = nexp * nn;
            for (int wi = tid; wi < work; wi += nt) {
                const int e_i = wi / nn, u = wi - e_i * nn;
                const int k = s_exp[e_i];
                Real Qx, Qy, Qz;
                load_q<Real>(cd, k, Qx, Qy, Qz);
                const NbrEntry<Real> e = s_nbr[u];
                const Real base = Qx * e.ax + Qy * e.ay + Qz * e.az - e.c0 - kq;
                if (test_cover<Real, MIXED>(base + drr * Qx - k1 * e.ax, (Real)0, cd, ri, roff_i, k, s_nbr_j[u], 0)) atomicAdd(&s_ev[3 * u + 0], -1);
                if (test_cover<Real, MIXED>(base + drr * Qy - k1 * e.ay, (Real)0, cd, ri, roff_i, k, s_nbr_j[u], 1)) atomicAdd(&s_ev[3 * u + 1], -1);
                if (test_cover<Real, MIXED>(base + drr * Qz - k1 * e.az, (Real)0, cd, ri, roff_i, k, s_nbr_j[u], 2)) atomicAdd(&s_ev[3 * u + 2], -1);
            }
            __syncthreads();
        }
        ncov = wave_sum_i(ncov);
        if ((tid & (WAVE - 1)) == 0) atomicAdd(&s_ncov, ncov);
        __syncthreads();

        // eq F_cav_patch: atom i gains G0_i ev / (N dr) per axis, neighbour j the opposite
        const long long qf = cd->qfix[ai];
        long long own0 = 0, own1 = 0, own2 = 0;
        for (int u = tid; u < nn; u += nt) {
            const int e0 = s_ev[3 * u], e1 = s_ev[3 * u + 1], e2 = s_ev[3 * u + 2];
            if (!(e0 | e1 | e2)) continue;
            const int aj = cd->s_idx[s_nbr_j[u]];
            if (e0) { const long long v = (long long)e0 * qf; own0 += v; atomicAdd((unsigned long long *)&cd->f_cav[3 * aj + 0], (unsigned long long)(-v)); }
            if (e1) { const long long v = (long long)e1 * qf; own1 += v; atomicAdd((unsigned long long *)&cd->f_cav[3 * aj + 1], (unsigned long long)(-v)); }
            if (e2) { const long long v = (long long)e2 * qf; own2 += v; atomicAdd((unsigned long long *)&cd->f_cav[3 * aj + 2], (unsigned long long)(-v)); }
        }
        if (own0) atomicAdd(&s_own[0], (unsigned long long)own0);
        if (own1) atomicAdd(&s_own[1], (unsigned long long)own1);
        if (own2) atomicAdd(&s_own[2], (unsigned long long)own2);
        __syncthreads();
        if (tid == 0) {
            for (int s = 0; s < 3; ++s)
                if (s_own[s]) atomicAdd((unsigned long long *)&cd->f_cav[3 * ai + s], s_own[s]);
            e_cav = cd->g0[ai] * (double)(N - s_ncov) / (double)N;  // eq G_cav_patch
            n_exp = (double)(N - s_ncov);
        }
    }
    if (tid == 0) {
        cd->f_pair[ai] = make_double4(pv[0], pv[1], pv[2], 0.0);
        cd->e_atom[ai] = make_double4(0.5 * pv[3], 0.5 * pv[4], e_cav, n_exp);
    }
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
    if (!cd->stats->active) return;
    __shared__ double s_w[ATOM_BLOCK / WAVE][WPART];
    const int lb = blockIdx.x - bt.blk_off[c];
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
    if (lb == 0 && threadIdx.x == 0) cd->stats->pending_post = 1;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_chain(const Batch &b, int do_post, int do_fk, hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chain, dim3(b.n_chains), dim3(CHAIN_THREADS), 0, s, b, do_post, do_fk);
    return hipGetLastError();
}

hipError_t launch_place(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_cellscan(const Batch &b, hipStream_t s)
{
    if (b.n_chains <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cellscan, dim3(b.n_chains), dim3(CHAIN_THREADS), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_scatter(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_rank(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rank, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_wrench(const Batch &b, hipStream_t s)
{
    if (b.total_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wrench, dim3(b.total_blocks), dim3(ATOM_BLOCK), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_force(const Batch &b, int precision, hipStream_t s)
{
    if (b.total_atoms <= 0) return hipSuccess;
    if (precision == 1)
        hipLaunchKernelGGL(k_force<float>, dim3(b.total_atoms), dim3(FORCE_THREADS), 0, s, b);
    else
        hipLaunchKernelGGL(k_force<double>, dim3(b.total_atoms), dim3(FORCE_THREADS), 0, s, b);
    return hipGetLastError();
}

}  // namespace kcm
