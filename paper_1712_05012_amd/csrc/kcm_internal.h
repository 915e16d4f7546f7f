// kcm_internal.h -- device-side layout of a chain and the launch interface
// between the host runtime (kcm_host.cpp) and the gfx950 kernels
// (kcm_kernels.hip).  Not part of the public ABI.
#pragma once

#include "../../include/kcm.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kcm {

constexpr int APR = 10;              // atoms per residue
constexpr int CHAIN_THREADS = 1024;  // one workgroup per chain: 16 waves
constexpr int SCAN_CHUNK = 4096;     // cells per workgroup of the cell-count scan
constexpr int SCAN_MAX_CHUNKS = 16384; // chunks per chain the scatter's offset table holds
constexpr int JOINT_BLOCK = 256;     // joints per workgroup of the torque / step / kinematics kernels
constexpr int MAX_NBR = KCM_NBR_CHUNK; // solvation neighbours of one atom kept in LDS (the list, its atoms
                                      // and its events, 6,720 bytes, let 24 waves share a CU)
constexpr int MAX_REACH = 3;         // cell-stencil half width the force kernel supports (cells >= reach/3)
constexpr double FIX_SCALE = 4294967296.0;  // fixed-point units per kcal/mol/A (2^32)
constexpr int WPART = 10;            // doubles per wrench partial: F(3), T(3), E(3), flag

// Per-chain scalars the kernels read and write (device memory).
struct ChainStats {
    double e_elec, e_vdw, e_cav;   // energies at the last force evaluation
    double max_tau, max_dtheta;    // of the last applied step
    double tol;                    // convergence threshold on max|dtheta| (<= 0: none)
    int64_t iterations;            // iterations applied since the chain was built
    int64_t iter_limit;            // stop when iterations reaches this (kcm_fold)
    double saved_tol;              // tol and iter_limit of before a kcm_fold call, restored at its end
    int64_t saved_limit;
    int32_t status;                // 0 ok, -4 numeric, -6 neighbour capacity
    int32_t converged;
    int32_t active;                // 0: the chain is stopped (converged, limit or failure)
    int32_t nbr_overflow;          // set by the force kernel, folded into status
    int32_t need_grid;             // 1: no bounding box of the current conformation yet
    int32_t pending_post;          // 1: forces of an iteration await their post phase
    int32_t post_bad;              // set by the torque kernel: a non-finite force in the pending post phase
    int32_t run;                   // 0: the kernels after the step skip this chain in this iteration
    int32_t grid_bad;              // this iteration's grid could not be sized: the chain stops
    int32_t pad;
    // Monte Carlo minimization: energies of the starting, accepted and lowest
    // states, completed and accepted trials, this trial's decisions
    double mc_e_start, mc_e_acc, mc_e_best;
    int64_t mc_trials, mc_accepted;
    int32_t mc_acc, mc_best;
};
// active is read by the torque and step kernels and written only at the end of
// an iteration (or call); run (set by the step) and grid_bad (set where the
// iteration's grid is sized, after the placement) are read by every later
// kernel.  So no kernel reads a flag that another workgroup of the same kernel
// may change, except grid_bad in the key kernel that sizes the grid in every
// workgroup: all of them reach the same decision.

// The cell grid of the current iteration (sized at its start from the last
// bounding box).
struct Grid {
    double origin[3];
    double cell, inv_cell;
    double reach_len;     // largest interaction distance (pair cutoff or solvation neighbour limit)
    int32_t dims[3];
    int32_t reach;        // stencil half width in cells
    int32_t n_cells;
    int32_t pad;
};

// Everything one chain owns on the device.  The struct itself lives at the
// start of the chain's device block; every pointer points into that block.
struct ChainDev {
    int32_t n_atoms, n_joints, n_links, n_samples;  // n_joints: the 2m backbone joints
    int32_t n_chi;       // side-chain joints (0 or m), stored after the backbone joints
    int32_t n_bb_blocks; // joint blocks of the backbone; the side-chain joints' blocks follow
    int32_t pad_chi[2];
    int32_t cap_cells, precision, terms, step_rule;
    double cutoff, kappa, max_step, diel_k, coulomb;  // coulomb = C / diel_k
    double w13, w14e, w14v, delta_r, r_probe, cell_min, roff_max;
    uint32_t m12[APR], m13[APR], m14[APR];  // bond classes per slot, bit (dres+1)*10 + slot_j
    uint32_t pad_masks[2];
    // the same classes as one word per slot: two bits at bit 2 ((dres+1)*10 + slot_j),
    // 0 none, 1 1-2, 2 1-3, 3 1-4 (m12 before m13 before m14); the (elec, vdw)
    // pair weights of each class in FP32 and FP64, and bit c set when both
    // weights of class c are zero
    uint64_t cls_word[APR];
    float wtab32[8];
    double wtab64[8];
    int32_t skip_cls32, skip_cls64;

    double *theta, *dtheta, *tau;
    double *mc_theta;    // [2][J]: accepted, then lowest angles of Monte Carlo minimization
    uint8_t *mask;
    double4 *joint0;     // [J][2]: (u0, 0), (p0, 0) zero-position axis and point
    double4 *jcur;       // [J][2]: current (u, 0), (p, 0)
    double *xform;       // [L][12] link transforms: R row-major, then t
    double *xform_loc;   // [J][12] product of the joint transforms from the start of j's joint block to j
    double *blk_xf;      // [nJB][12] product of all joint transforms of each joint block
    double *tmax_part;   // [nJB] max |tau| over the masked joints of each joint block
    int32_t *bad_part;   // [nJB] 1 if a torque of the block is not finite
    double4 *r0;         // [n] zero-position coordinates
    double4 *r;          // [n] current coordinates
    double4 *aparam;     // [n] (q, R_vdw, sqrt(eps), R_off)
    double *g0;          // [n] 4 pi gamma R_off^2
    long long *qfix;     // [n] event quantum G0/(N dr) in fixed point
    int32_t *cell_key;   // [n] cell of each atom
    int32_t *cell_count; // [cap] atoms per cell (zero between iterations)
    int32_t *cell_start; // [cap+1] cell starts in the cell-ordered arrays
    int32_t *cell_local; // [cap] exclusive scan of the counts inside each chunk of SCAN_CHUNK cells
    int32_t *scan_part;  // [cap / SCAN_CHUNK, rounded up] cell count of each chunk
    double *bbox_part;   // [blocks][6] per-workgroup min xyz, max xyz of the placed atoms
    double *wrench_part; // [blocks][WPART] per-workgroup wrench (F, r x F), energies, failure flag
    double4 *s_r;        // [n] positions in cell order
    double4 *s_p;        // [n] parameters in cell order
    int32_t *s_tmp;      // [n] scatter order (before the stable rank)
    int32_t *s_idx;      // [n] atom of each sorted slot (the cell order)
    double4 *f_pair;     // [n] Coulomb + LJ force
    long long *f_cav;    // [3n] solvation force, fixed point
    double4 *e_atom;     // [n] (elec, vdw, cav, exposed samples) per atom
    double4 *q64;        // [N] unit sample directions
    float4 *q32;         // [N]
    Grid *grid;          // grid of the current iteration
    ChainStats *stats;
};

// The chains of one call.  table: device array of device descriptors;
// atom_off / blk_off / jblk_off: device arrays [n_chains+1] of cumulative atom
// counts, of cumulative per-atom workgroup counts (ATOM_BLOCK atoms per
// workgroup) and of cumulative joint-block counts (JOINT_BLOCK joints each).
constexpr int ATOM_BLOCK = 256;
struct Batch {
    ChainDev *const *table;
    const int32_t *atom_off;
    const int32_t *blk_off;
    const int32_t *jblk_off;
    const int32_t *scan_off;  // cumulative count of SCAN_CHUNK-cell chunks of the chains' capacities
    int n_chains;
    int total_atoms;
    int total_blocks;
    int total_jblocks;
    int total_scan_blocks;
    int max_scan_chunks;      // most chunks of one chain (sizes the chunk-offset table in LDS)
};

// Modes of the step/kinematics and placement kernels.
enum : int { MODE_ITER = 0, MODE_FINAL = 1, MODE_BOOT = 2 };

// Launchers (kcm_kernels.hip).  One iteration is
//   tau, stepfk (post phase of the previous forces if pending, then the
//   kinematics of each joint block), place, cellkey (the grid of the placed
//   conformation, keys and counts), cellscan, scatter, rank, force, wrench;
// a call ends with tau, stepfk(MODE_FINAL), finish.  A chain without a grid
// (new, or new angles) first runs stepfk(MODE_BOOT), place(MODE_BOOT), gridboot.
hipError_t launch_tau(const Batch &b, hipStream_t s);
hipError_t launch_stepfk(const Batch &b, int mode, hipStream_t s);
hipError_t launch_gridboot(const Batch &b, hipStream_t s);
hipError_t launch_finish(const Batch &b, hipStream_t s);
hipError_t launch_place(const Batch &b, int mode, hipStream_t s);
hipError_t launch_cellkey(const Batch &b, hipStream_t s);
hipError_t launch_cellscan(const Batch &b, hipStream_t s);
hipError_t launch_scatter(const Batch &b, hipStream_t s);
constexpr int FORCE_SHAPE_COUNT = 4;  // launch shapes of the force kernel (kcm_set_force_variant)
hipError_t launch_force(const Batch &b, int precision, int shape, hipStream_t s);
hipError_t launch_rank(const Batch &b, hipStream_t s);
hipError_t launch_wrench(const Batch &b, hipStream_t s);
constexpr int FOLD_BEGIN = 0, FOLD_END = 1;
constexpr int MC_RESET = 0, MC_PROPOSE = 1;  // k_mc_propose: flags only, or flags and new angles
constexpr int MC_INIT = 0, MC_TRIAL = 1;     // k_mc_decide: take the state, or the Metropolis test
hipError_t launch_mc_propose(const Batch &b, int mode, const double *delta, const int64_t *delta_off, int trial,
                             hipStream_t s);
hipError_t launch_mc_decide(const Batch &b, int mode, const double *u, int n_trials, int trial, double kT,
                            hipStream_t s);
hipError_t launch_mc_apply(const Batch &b, hipStream_t s);
hipError_t launch_set_theta(const Batch &b, const double *theta, const int64_t *theta_off, hipStream_t s);
hipError_t launch_stats_gather(const Batch &b, ChainStats *out, hipStream_t s);
hipError_t launch_fold_control(const Batch &b, int mode, double tol, int64_t max_iter, hipStream_t s);

}  // namespace kcm
