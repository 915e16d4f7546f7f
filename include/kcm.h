/*
 * kcm.h -- C ABI of libkcm, the gfx950 (MI355X) implementation of one
 * iteration of the kinetostatic compliance method (KCM) of Protofold II
 * (Tavousi, Behandish, Ilies, Kazerounian): forward kinematics, a cell list,
 * Coulomb + Lennard-Jones + SASA-enumeration solvation forces, Jacobian-
 * transpose joint torques and the compliance step.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Units: Angstrom, elementary charge, kcal/mol, radian.  Torque is in
 *    kcal/mol per radian, kappa in radian per (kcal/mol).
 *  * A chain of m residues has n = 10 m atoms, J = 2 m joints and 2 m + 1
 *    links.  Atom 10 i + s is slot s of residue i, slots in the order
 *    N, H, CA, HA, CB, HB1, HB2, HB3, C, O.  Joint 2 i is phi_i (axis N_i->CA_i),
 *    joint 2 i + 1 is psi_i (axis CA_i->C_i); joint j turns every atom of the
 *    links after it (Sec. 2.1, Table 2).  omega is fixed at 180 degrees.  A
 *    chain built with side chains has J = 3 m: joint 2 m + i is chi_i, which
 *    turns HB1..HB3 of residue i about CA_i->CB_i.
 *  * Angles theta are the dihedrals phi/psi themselves, in (-pi, pi]; the zero
 *    position (ZP) of the paper's ZRPD convention is phi = psi = 180 degrees.
 *  * Host pointers are read during the call and not kept.  Device memory is
 *    owned by the caller: kcm_build_chain lays a chain out inside the block it
 *    is given and never frees it.  The one exception is per-call bookkeeping:
 *    kcm_step, kcm_fold, kcm_mc_minimize and kcm_set_theta_batch keep, per
 *    (device, stream), a device table of the chain set (descriptor pointers
 *    and four offset arrays, about 24 bytes per chain), the gathered per-chain
 *    records (device and pinned host) and the captured HIP graphs; these are
 *    allocated when a larger set first arrives, reused while the set is
 *    unchanged (graphs are dropped when one of their chains is freed) and
 *    kept until the process ends.  kcm_step_noalloc takes the same
 *    bookkeeping from static device memory and allocates nothing.
 *    Host-side handles are owned by the library (kcm_chain_free).  hip_stream
 *    is a hipStream_t (NULL = default stream); work is queued asynchronously
 *    unless a function says it synchronises.
 *  * Every function returns a kcm_status; no exception crosses the ABI.  The
 *    calling thread's last error message is available from kcm_last_error().
 *  * The entry points that launch work (kcm_step, kcm_fold, kcm_mc_minimize)
 *    may be called from several threads; the library serialises them, each
 *    for the whole of its call.
 *  * A numeric failure (NaN/Inf in forces or torques) marks only the chain it
 *    occurs in: its theta is left unchanged, its report carries
 *    KCM_E_NUMERIC, and the other chains of a batched call continue.
 */
#ifndef KCM_H
#define KCM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KCM_OK = 0,
    KCM_E_INVAL = -1,    /* bad argument */
    KCM_E_NOMEM = -2,    /* the given device block is too small */
    KCM_E_DEVICE = -3,   /* a HIP runtime call failed */
    KCM_E_NUMERIC = -4,  /* NaN/Inf in this chain's forces or torques */
    KCM_E_STATE = -5,    /* call not valid in the handle's current state */
    KCM_E_CAPACITY = -6  /* an atom has 131072 or more solvation neighbours (the force
                            kernel takes any smaller count, in LDS chunks of
                            KCM_NBR_CHUNK) */
} kcm_status;

/* Solvation neighbours of one atom that the force kernel holds in LDS at once;
 * an atom with more is processed in chunks of this many (same results). */
#define KCM_NBR_CHUNK 240

enum { KCM_STEP_CAPPED = 0, KCM_STEP_PAPER = 1, KCM_STEP_LINEAR = 2 };
enum { KCM_FP64 = 0, KCM_MIXED = 1 };
enum { KCM_TERM_ELEC = 1, KCM_TERM_VDW = 2, KCM_TERM_CAV = 4, KCM_TERM_ALL = 7 };

/* Force-field inputs of one residue type, per atom slot (slot order above). */
typedef struct {
    double q[10];          /* partial charge, e */
    double sigma[10];      /* Lennard-Jones sigma, A; vdW radius R = 2^(1/6) sigma / 2 */
    double eps[10];        /* Lennard-Jones well depth, kcal/mol */
    double hydrophobicity; /* residue hydrophobicity; gamma = g_hydro * hydrophobicity */
} kcm_residue_type;

/* What defines one chain (the paper's Fig. 5 steps 1-3 and user options). */
typedef struct {
    int32_t n_res;                  /* m >= 1 */
    const int32_t *res_type;        /* [m], values in 0 .. n_types-1 */
    const kcm_residue_type *types;  /* [n_types] */
    int32_t n_types;
    const double *theta0;           /* [J] initial phi_1, psi_1, ..., phi_m, psi_m, then chi_1 .. chi_m
                                       with side chains; NULL = ZP (phi = psi = 180, chi = 60 degrees) */
    const uint8_t *joint_mask;      /* [J] 0 = joint held fixed (Sec. 4.1 options); NULL = all free */
    int32_t side_chains;            /* 0: J = 2m backbone joints.  1: J = 3m, with one side-chain
                                       joint per residue (Sec. 2.1): chi_i = dihedral N-CA-CB-HB1,
                                       turning HB1..HB3 about the CA->CB bond */
} kcm_chain_desc;

/* Method parameters.  kcm_default_params() fills the defaults listed here. */
typedef struct {
    double cutoff;      /* 10.0  Coulomb and LJ cutoff, pairs with d <= cutoff count (eqs 02_2, 03_2) */
    double kappa;       /* 1e-3  compliance, rad per kcal/mol (eq KCM_07) */
    double max_step;    /* 1e-3  s: the largest joint step of the PAPER and CAPPED rules, rad */
    int32_t step_rule;  /* KCM_STEP_CAPPED: kappa tau min(1, s/(kappa |tau|max));
                           KCM_STEP_PAPER: s tau/|tau|max (eq KCM_07); KCM_STEP_LINEAR: kappa tau */
    int32_t precision;  /* KCM_FP64, or KCM_MIXED: FP32 pair and sample tests (FP64 recheck near
                           ties), FP64 kinematics, torques and step */
    int32_t terms;      /* KCM_TERM_* bitmask; ELEC and VDW go together */
    int32_t n_orbits;   /* 14 -> N = 250 samples per offset sphere (Sec. 3.4) */
    double diel_k;      /* 4.0   distance-dependent dielectric eps = diel_k * d (Sec. 2.2) */
    double w13;         /* 0.0   weight of 1-3 pairs (1-2 pairs are always 0) (eqs 03_8, 03_9) */
    double w14_elec;    /* 1/1.2 Coulomb weight of 1-4 pairs */
    double w14_vdw;     /* 0.5   LJ weight of 1-4 pairs */
    double delta_r;     /* 0.05  finite difference of eq (finitediff), A */
    double r_probe;     /* 1.4   water probe radius added to R (Sec. 2.2) */
    double g_hydro;     /* 0.025 kcal/mol/A^2 per unit hydrophobicity */
    double cell_size;   /* 0 = automatic (cutoff / 2, coarsened when the grid exceeds its capacity) */
} kcm_params;

/* Per chain, after a kcm_step call: values of the chain's last iteration. */
typedef struct {
    double e_elec, e_vdw, e_cav; /* energies of the conformation the forces were taken at */
    double max_tau;              /* max |tau| over free joints */
    double max_dtheta;           /* max |dtheta| applied */
    int64_t iterations;          /* iterations applied to this chain since it was built */
    int32_t status;              /* KCM_OK, KCM_E_NUMERIC or KCM_E_CAPACITY */
    int32_t converged;           /* 1 once max|dtheta| < tol under kcm_fold */
} kcm_step_report;

typedef struct {
    int64_t iterations;  /* iterations run by this call */
    int32_t converged;   /* max|dtheta| < tol reached */
    int32_t status;
    double seconds;      /* wall time of the call */
} kcm_fold_result;

/* Per chain result of kcm_mc_minimize. */
typedef struct {
    double e_start;      /* energy (the chain's terms) of its angles at the start of the call */
    double e_accepted;   /* energy of the accepted state at the end */
    double e_best;       /* lowest energy of any state evaluated in the call */
    int64_t trials;      /* completed trials */
    int64_t accepted;    /* accepted trials */
    int32_t status;
    int32_t pad;
} kcm_mc_result;

typedef struct kcm_chain kcm_chain;

/* Fill *p with the defaults above. */
void kcm_default_params(kcm_params *p);

/* Bytes of caller-owned device memory a chain needs (256-byte aligned block):
 * the per-joint state of the kinematic chain (Sec. 2.1, Fig. 5), per-atom
 * positions, parameters and forces (Secs. 2.2 and 3.4), the cell grid of
 * Sec. 3.2 (capacity max(8192, 8n) cells) and the offset-sphere samples of
 * Sec. 3.4.  Depends on n_res, desc->side_chains and params->n_orbits only.
 * KCM_E_INVAL for a NULL argument or inputs kcm_build_chain would reject
 * (n_res outside 1 .. 524288, bad parameters). */
kcm_status kcm_chain_bytes(const kcm_chain_desc *desc, const kcm_params *params, size_t *bytes);

/* Build a chain (Fig. 5 steps 1-3): zero-position geometry from the residue
 * template, bond-path interaction classes (Sec. 3.3), per-atom parameters, the
 * offset-sphere sample set, and theta0.  Lays everything out in dev_mem (at
 * least kcm_chain_bytes bytes, device memory of the current device) with
 * asynchronous copies on hip_stream and returns a host handle in *out.
 * Errors: KCM_E_INVAL (bad desc/params, dev_mem not 256-byte aligned or not
 * device memory), KCM_E_NOMEM (bytes too small), KCM_E_DEVICE. */
kcm_status kcm_build_chain(const kcm_chain_desc *desc, const kcm_params *params, void *dev_mem,
                           size_t bytes, void *hip_stream, kcm_chain **out);

/* Run n_iter KCM iterations on each of n_chains chains (Fig. 5 steps 4-8):
 * forward kinematics (eqs kin_02-kin_04, r1), cell list (Sec. 3.2), pair and
 * solvation forces (eqs 02-04_3, G_cav_patch, F_cav_patch, finitediff,
 * Algorithm 1), link wrenches and joint torques (eqs KCM_01-KCM_06, row scan
 * of eq 04_9), and the compliance step (eq KCM_07).  All chains of one call
 * must share precision and live on the current device; the chains are
 * processed together in one set of launches per iteration.  Chains already
 * converged under kcm_fold are skipped.  If reports != NULL the call
 * synchronises hip_stream and fills reports[n_chains]; otherwise it only
 * queues work.  Returns KCM_E_NUMERIC / KCM_E_CAPACITY if any chain reported
 * it (the other chains are still advanced). */
kcm_status kcm_step(kcm_chain *const *chains, int n_chains, int n_iter, void *hip_stream,
                    kcm_step_report *reports);

/* kcm_step for callers that cannot allocate memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same
 * iterations, results (bit for bit) and reports as kcm_step, with these
 * differences:
 *  * the call allocates nothing, on the device or the host: the batch table
 *    and the gathered report records live in a file-scope device array of
 *    the library (at most KCM_NOALLOC_SCRATCH_BYTES per device, held until
 *    the process ends);
 *  * at most KCM_NOALLOC_MAX_CHAINS chains per call (more: KCM_E_INVAL);
 *  * kernels are launched directly (no HIP graphs; kcm_set_graphs and
 *    kcm_set_timing do not apply);
 *  * every call on one device shares that device's array.  The library
 *    orders its own calls: a call with a different chain set, or from another
 *    stream, first waits for the previous call's stream.  Work that the
 *    caller queues around the calls and that depends on their order is the
 *    caller's to order; calls from different processes use different arrays.
 * If reports != NULL the call synchronises hip_stream and fills
 * reports[n_chains].  Errors: those of kcm_step, KCM_E_INVAL for more than
 * KCM_NOALLOC_MAX_CHAINS chains or a device index above 63. */
#define KCM_NOALLOC_MAX_CHAINS 1024
#define KCM_NOALLOC_SCRATCH_BYTES 262144
kcm_status kcm_step_noalloc(kcm_chain *const *chains, int n_chains, int n_iter, void *hip_stream,
                            kcm_step_report *reports);

/* Iterate every chain until max|dtheta| < tol_dtheta or max_iter iterations
 * (Fig. 5 step 9); convergence is polled every check_every iterations (>= 1).
 * For the call, tol_dtheta and max_iter replace each chain's own stopping
 * rule (kcm_set_limits); the call puts that rule back at its end, so a chain
 * that has reached its own iteration cap stays stopped afterwards.
 * Synchronises hip_stream.  results[n_chains] may be NULL.  Errors:
 * KCM_E_INVAL (max_iter < 0, check_every < 1, or the chain-set errors of
 * kcm_step), KCM_E_DEVICE; otherwise the first failing chain's status. */
kcm_status kcm_fold(kcm_chain *const *chains, int n_chains, double tol_dtheta, int max_iter,
                    int check_every, void *hip_stream, kcm_fold_result *results);

/* Monte Carlo minimization: the hybrid of Monte Carlo sampling and steepest
 * descent listed among the search improvements of Sec. 4, in the form of Li
 * and Scheraga (Monte Carlo minimization) with the Metropolis rule.  The
 * start is each chain's current angles and their energy E (the chain's terms:
 * Coulomb + LJ, plus solvation when enabled).  Trial k of chain c:
 *   theta' = wrap(accepted + delta) on the free joints (mask 1),
 *   then n_descent KCM iterations from theta' (the chain's step rule),
 *   E' = energy of the reached angles (one more evaluation),
 *   accepted when E' <= E or u < exp(-(E' - E)/kT) (kT = 0: downhill only).
 * delta: DEVICE array, the chains' blocks [n_trials][J_c] one after the other
 * in call order (radians); u: DEVICE array [n_chains][n_trials], uniform in
 * [0, 1).  Both are read during the call only; pageable host memory is
 * rejected with KCM_E_INVAL.  All trials of all chains run
 * on the device with no host round trip.  Afterwards each chain holds its
 * accepted angles (kcm_mc_best_theta gives the lowest); its positions and
 * forces are those of the last evaluated trial, and its next kcm_step starts
 * with a fresh grid.  A chain that fails numerically keeps the accepted
 * angles of before the failure.  The call clears the chains' convergence
 * tolerance and iteration limit (kcm_set_limits), so every descent runs its
 * n_descent iterations.  results[n_chains] may be NULL.
 * Synchronises hip_stream.  Errors: KCM_E_INVAL (negative n_trials or
 * n_descent, kT < 0 or NaN, a missing or non-device delta/u, or the chain-set
 * errors of kcm_step), KCM_E_DEVICE; otherwise the first failing chain's
 * status, as kcm_step. */
kcm_status kcm_mc_minimize(kcm_chain *const *chains, int32_t n_chains, int32_t n_trials, int32_t n_descent,
                           double kT, const double *delta, const double *u, void *hip_stream,
                           kcm_mc_result *results);

/* The lowest-energy angles (host array [J]) of the chain's last
 * kcm_mc_minimize call; synchronises hip_stream. */
kcm_status kcm_mc_best_theta(const kcm_chain *chain, void *hip_stream, double *theta);

/* Copy a chain's state to host arrays (any pointer may be NULL); synchronises
 * hip_stream.  theta[J] and dtheta[J] (the angles and the last applied step of
 * eq KCM_07); xyz[n][3] and force[n][3] (total, eqs 02, 03 and F_cav_patch) at
 * the conformation of the last force evaluation; tau[J] (eqs KCM_01-KCM_06).
 * The angles are the whole state a chain carries from one iteration to the
 * next: a chain built from them continues bit for bit. */
kcm_status kcm_get_state(const kcm_chain *chain, void *hip_stream, double *theta, double *xyz,
                         double *force, double *tau, double *dtheta);

/* Per-term forces of the last evaluation: pair (Coulomb + LJ) and solvation,
 * host arrays [n][3]; synchronises hip_stream. */
kcm_status kcm_get_forces(const kcm_chain *chain, void *hip_stream, double *f_pair, double *f_cav);

/* Per-atom terms of the last evaluation, host arrays [n] (any may be NULL):
 * Coulomb and LJ energy (half of every pair the atom is in), solvation energy
 * G0_i f_i (eq G_cav_patch) and the number of exposed samples N f_i (-1 when
 * the solvation term is off).  Synchronises hip_stream. */
kcm_status kcm_get_atom_terms(const kcm_chain *chain, void *hip_stream, double *e_elec, double *e_vdw,
                              double *e_cav, int32_t *n_exposed);

/* Per-chain stopping rule applied inside kcm_step: once max|dtheta| of an
 * iteration is below tol_dtheta (tol_dtheta <= 0: never) or the chain has run
 * max_iterations iterations since it was built (<= 0: no cap), the chain is
 * marked converged / finished and later launches skip it.  Its reports then
 * carry converged = 1 or iterations == max_iterations.  Used by serving loops
 * that advance many chains with one call (Fig. 5 step 9, per chain).  A
 * kcm_fold call suspends the rule for its duration and restores it;
 * kcm_mc_minimize clears it.  Synchronises hip_stream.  Errors: KCM_E_INVAL
 * (null chain, tol_dtheta not finite), KCM_E_DEVICE. */
kcm_status kcm_set_limits(kcm_chain *chain, double tol_dtheta, int64_t max_iterations, void *hip_stream);

/* Replace a chain's theta (host array [J]), e.g. to resume from a checkpoint
 * or to re-synchronise with a reference; clears its converged flag. */
kcm_status kcm_set_theta(kcm_chain *chain, const double *theta, void *hip_stream);

/* kcm_set_theta for many chains from one DEVICE array: chain c's J_c angles
 * follow the earlier chains' in call order.  Angles are wrapped into
 * (-pi, pi] on the device; they must be finite (a non-finite angle makes the
 * chain fail with KCM_E_NUMERIC at its next iteration); pageable host memory
 * is rejected with KCM_E_INVAL.  Each chain's flags
 * are cleared as by kcm_set_theta.  The array is read by work queued on
 * hip_stream, so it must stay valid until that work has run (the next
 * kcm_step on the stream suffices). */
kcm_status kcm_set_theta_batch(kcm_chain *const *chains, int32_t n_chains, const double *theta,
                               void *hip_stream);

/* The cell list of the last evaluation (Sec. 3.2): dims[3] cells per axis,
 * *cell_size (A), origin[3] (grid corner), order[n] (atom index of each
 * sorted slot), cell_start[dims0*dims1*dims2 + 1].  Any pointer may be NULL;
 * *n_cells receives the cell count.  Synchronises hip_stream. */
kcm_status kcm_get_cells(const kcm_chain *chain, void *hip_stream, int32_t *dims, double *cell_size,
                         double *origin, int32_t *n_cells, int32_t *order, int32_t *cell_start,
                         int32_t cell_start_capacity);

/* Sizes of a built chain: atoms, joints J (2m, or 3m with side chains),
 * offset-sphere samples and the precision. */
kcm_status kcm_chain_info(const kcm_chain *chain, int32_t *n_atoms, int32_t *n_joints,
                          int32_t *n_samples, int32_t *precision);

/* Optional per-kernel timing with hipEvents on the launch stream: when
 * every > 0, kcm_step records an event pair around the force kernel and one
 * around the whole iteration on every every-th iteration (a sample, so that
 * the events barely perturb the timeline); every = 0 switches it off.
 * kcm_get_timing returns the summed milliseconds and sample counts of the
 * force kernel and of the iteration since the last reset (synchronises every
 * stream it recorded on). */
kcm_status kcm_set_timing(int every);
/* Launch mode of kcm_step (process-wide): iterations >= 1 (default 1)
 * captures that many consecutive iterations of a call's chains as one HIP
 * graph (on a private stream, once per batch composition and depth) and
 * replays it on hip_stream, with single-iteration replays for the rest of a
 * call; iterations = 0 launches the kernels directly.  Every mode gives
 * identical results.  KCM_E_INVAL unless 0 <= iterations <= 64. */
kcm_status kcm_set_graphs(int iterations);

/* Launch shape of the force kernel (process-wide), for the autotuner:
 * 0 (default): each lane loads two candidates per trip of the candidate loop,
 * and step 1 reads the solvation neighbours in blocks of 4 before it checks
 * which sample slots are done; 1: one candidate per trip, blocks of 4;
 * 2: as 1, and 3: as 0, with the atoms handed to the 8 XCDs in contiguous
 * eighths (XCD-aware order).  Every shape gives identical
 * results (the same visiting order and decisions).  Graphs captured in
 * another shape are captured again.  KCM_E_INVAL unless
 * 0 <= variant < KCM_FORCE_VARIANTS. */
#define KCM_FORCE_VARIANTS 4
kcm_status kcm_set_force_variant(int variant);

kcm_status kcm_get_timing(double *force_ms, int64_t *force_launches, double *iter_ms,
                          int64_t *iterations, int reset);

/* Release a handle (not the device block). */
kcm_status kcm_chain_free(kcm_chain *chain);

/* Message of the calling thread's last failing call ("" if none). */
const char *kcm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KCM_H */
