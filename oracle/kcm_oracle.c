/*
 * kcm_oracle.c -- plain FP64 CPU oracle for one iteration of the kinetostatic
 * compliance method (KCM) of Protofold II (Tavousi, Behandish, Ilies,
 * Kazerounian).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; the two meet only
 * in the seeded input arrays.
 *
 * Every routine is written from the paper's definitions, slowly and in the
 * paper's order:
 *   zero position + links ....... Sec. 2.1 (kinematic model, Tables 1-2, ZRPD)
 *   forward kinematics .......... eqs (kin_02)-(kin_04), (r1); Sec. 3.1
 *   bond graph + weights ........ Sec. 3.3 (bonds tree), eqs (03_8)-(03_9)
 *   Coulomb + Lennard-Jones ..... eqs (02), (02_1), (02_2), (03), (03_1), (03_2)
 *   solvation (SASA) ............ eqs (04), (04_2), (G_cav_patch),
 *                                 (F_cav_patch), (finitediff); Algorithm 1 and
 *                                 the C-state rules of Sec. 3.4
 *   link wrench + joint torque .. eqs (KCM_01), (KCM_02), (KCM_04)-(KCM_06)
 *   compliance step ............. eq (KCM_07); Sec. 3.1 angle update
 *
 * Readings where the paper is silent or garbled (each one is listed in the
 * design notes of the repository):
 *   - dielectric: eps_ij = k_d * d (distance-dependent, k_d = 4), so
 *     E = C q_i q_j w / (k_d d^2) and the force is its exact gradient;
 *   - energies sum unordered pairs i<j once, so F = -grad E exactly;
 *   - one hard cutoff d <= r_cut for Coulomb and LJ;
 *   - 1-2 and 1-3 pairs have weight w13 (default 0), 1-4 pairs w14_elec,
 *     w14_vdw (defaults 1/1.2 and 1/2), all other pairs 1;
 *   - LJ well distance D_ij = R_i + R_j with R = 2^(1/6) sigma / 2;
 *   - SASA: no early exit after the first critical neighbour of an exposed
 *     sample, because eq (finitediff) defines f_{i,j,s} for every j on its own;
 *   - a sample is covered when ||q - r_j|| <= R_off_j (closed ball);
 *   - joint torque tau_k = u_k . sum_{a downstream of k} (r_a - p_k) x F_a;
 *   - step rules PAPER / LINEAR / CAPPED (see or_step).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC -o liboracle.so kcm_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846
#define OR_COULOMB 332.0636 /* kcal A / (mol e^2) */
#define APR 10              /* atoms per residue in the ZP template */

/* atom slots of one residue, in storage (= link) order */
enum { A_N = 0, A_H, A_CA, A_HA, A_CB, A_HB1, A_HB2, A_HB3, A_C, A_O };

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static void v_sub(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double v_dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void v_cross(const double *a, const double *b, double *o)
{
    double t0 = a[1] * b[2] - a[2] * b[1];
    double t1 = a[2] * b[0] - a[0] * b[2];
    double t2 = a[0] * b[1] - a[1] * b[0];
    o[0] = t0; o[1] = t1; o[2] = t2;
}
static double v_norm(const double *a) { return sqrt(v_dot(a, a)); }
static void v_unit(const double *a, double *o) { double n = v_norm(a); o[0] = a[0] / n; o[1] = a[1] / n; o[2] = a[2] / n; }
static double deg(double x) { return x * OR_PI / 180.0; }

/* 3x3 row-major matrices */
static void m_mul(const double *A, const double *B, double *C)
{
    double T[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            T[3 * r + c] = A[3 * r] * B[c] + A[3 * r + 1] * B[3 + c] + A[3 * r + 2] * B[6 + c];
    memcpy(C, T, sizeof T);
}
static void m_vec(const double *A, const double *x, double *y)
{
    double t0 = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    double t1 = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    double t2 = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
    y[0] = t0; y[1] = t1; y[2] = t2;
}
/* rotation by angle a about unit axis u, right-hand rule (Rodrigues) */
static void m_rot(const double *u, double a, double *R)
{
    double c = cos(a), s = sin(a), t = 1.0 - c;
    R[0] = c + u[0] * u[0] * t;        R[1] = u[0] * u[1] * t - u[2] * s; R[2] = u[0] * u[2] * t + u[1] * s;
    R[3] = u[1] * u[0] * t + u[2] * s; R[4] = c + u[1] * u[1] * t;        R[5] = u[1] * u[2] * t - u[0] * s;
    R[6] = u[2] * u[0] * t - u[1] * s; R[7] = u[2] * u[1] * t + u[0] * s; R[8] = c + u[2] * u[2] * t;
}

/* Place d so that |d-c| = bond, angle(b,c,d) = ang, dihedral(a,b,c,d) = tor. */
static void place(const double *a, const double *b, const double *c, double bond, double ang, double tor, double *d)
{
    double bc[3], ab[3], n[3], m[3];
    v_sub(c, b, bc); v_unit(bc, bc);
    v_sub(b, a, ab);
    v_cross(ab, bc, n); v_unit(n, n);
    v_cross(n, bc, m);
    double x = -bond * cos(ang), y = bond * sin(ang) * cos(tor), z = bond * sin(ang) * sin(tor);
    for (int k = 0; k < 3; ++k) d[k] = c[k] + x * bc[k] + y * m[k] + z * n[k];
}

/* ------------------------------------------------------------------ */
/* Chain topology and zero position (Sec. 2.1)                          */
/* ------------------------------------------------------------------ */
/* Residue i (0-based) holds atoms 10i..10i+9 in the slot order above.
 * Joints: 2i = phi_i (axis N_i -> CA_i, point N_i), 2i+1 = psi_i (axis CA_i -> C_i,
 * point CA_i).  Links: 0 = {N_0, H_0}; 2i+1 = {CA, HA, CB, HB1-3} of residue i;
 * 2i+2 = {C_i, O_i, N_{i+1}, H_{i+1}} (the last one {C, O}).  Joint j moves links
 * j+1 .. 2m.  ZP: phi = psi = omega = 180 deg, N_0 at the origin. */

int or_sizes(int m, int *n_atoms, int *n_joints, int *n_links)
{
    if (m < 1) return -1;
    *n_atoms = APR * m; *n_joints = 2 * m; *n_links = 2 * m + 1;
    return 0;
}

int or_link_of_atom(int a)
{
    int i = a / APR, s = a % APR;
    if (s <= A_H) return 2 * i;          /* N, H ride on the previous psi link (link 0 for i=0) */
    if (s <= A_HB3) return 2 * i + 1;    /* CA side */
    return 2 * i + 2;                    /* C, O */
}

/* Idealised geometry: bond lengths and angles named by the workload recipe,
 * tetrahedral 109.5 deg at CA and CB, amide H in the peptide plane. */
int or_build_zp(int m, double *r0 /* [10m][3] */)
{
    const double b_NCA = 1.458, b_CAC = 1.525, b_CN = 1.329, b_CO = 1.231, b_NH = 1.01, b_CH = 1.09, b_CACB = 1.53;
    const double a_NCAC = deg(111.2), a_CACN = deg(116.2), a_CNCA = deg(121.7), a_CACO = deg(120.8);
    const double a_CANH = deg(0.5 * (360.0 - 121.7)), a_tet = deg(109.5);
    double *R = r0;
    double *N0 = R + 3 * A_N, *CA0 = R + 3 * A_CA, *C0 = R + 3 * A_C;
    N0[0] = N0[1] = N0[2] = 0.0;
    CA0[0] = b_NCA; CA0[1] = 0.0; CA0[2] = 0.0;
    C0[0] = CA0[0] - b_CAC * cos(a_NCAC); C0[1] = b_CAC * sin(a_NCAC); C0[2] = 0.0;
    for (int i = 0; i < m; ++i) {
        double *N = R + 3 * (APR * i + A_N), *CA = R + 3 * (APR * i + A_CA), *C = R + 3 * (APR * i + A_C);
        if (i > 0) {
            const double *Np = R + 3 * (APR * (i - 1) + A_N), *CAp = R + 3 * (APR * (i - 1) + A_CA), *Cp = R + 3 * (APR * (i - 1) + A_C);
            place(Np, CAp, Cp, b_CN, a_CACN, deg(180.0), N);   /* psi_{i-1} = 180 */
            place(CAp, Cp, N, b_NCA, a_CNCA, deg(180.0), CA);  /* omega = 180 */
            place(Cp, N, CA, b_CAC, a_NCAC, deg(180.0), C);    /* phi_i = 180 */
        }
        place(C, CA, N, b_NH, a_CANH, 0.0, R + 3 * (APR * i + A_H));
        place(C, N, CA, b_CACB, a_tet, deg(-120.0), R + 3 * (APR * i + A_CB));
        place(C, N, CA, b_CH, a_tet, deg(120.0), R + 3 * (APR * i + A_HA));
        const double *CB = R + 3 * (APR * i + A_CB);
        place(N, CA, CB, b_CH, a_tet, deg(60.0), R + 3 * (APR * i + A_HB1));
        place(N, CA, CB, b_CH, a_tet, deg(180.0), R + 3 * (APR * i + A_HB2));
        place(N, CA, CB, b_CH, a_tet, deg(-60.0), R + 3 * (APR * i + A_HB3));
        place(N, CA, C, b_CO, a_CACO, 0.0, R + 3 * (APR * i + A_O));  /* anti to N_{i+1} */
    }
    return 0;
}

/* Covalent bonds of the chain (Sec. 3.3); returns the count, writes pairs if out != NULL. */
int or_bonds(int m, int *out /* [2*count] */)
{
    static const int intra[9][2] = {{A_N, A_H}, {A_N, A_CA}, {A_CA, A_HA}, {A_CA, A_CB}, {A_CA, A_C},
                                    {A_CB, A_HB1}, {A_CB, A_HB2}, {A_CB, A_HB3}, {A_C, A_O}};
    int k = 0;
    for (int i = 0; i < m; ++i) {
        for (int b = 0; b < 9; ++b) {
            if (out) { out[2 * k] = APR * i + intra[b][0]; out[2 * k + 1] = APR * i + intra[b][1]; }
            ++k;
        }
        if (i + 1 < m) {
            if (out) { out[2 * k] = APR * i + A_C; out[2 * k + 1] = APR * (i + 1) + A_N; }
            ++k;
        }
    }
    return k;
}

/* Per-atom force-field inputs from the residue-type tables.
 * R (vdW radius) = 2^(1/6) sigma / 2; gamma = g_hydro * hydrophobicity(residue). */
int or_atom_params(int m, const int *res_type, const double *type_q, const double *type_sigma,
                   const double *type_eps, const double *type_hydro, double g_hydro,
                   double *q, double *R, double *eps, double *gamma)
{
    const double k6 = pow(2.0, 1.0 / 6.0);
    for (int i = 0; i < m; ++i) {
        int t = res_type[i];
        for (int s = 0; s < APR; ++s) {
            int a = APR * i + s;
            q[a] = type_q[APR * t + s];
            R[a] = 0.5 * k6 * type_sigma[APR * t + s];
            eps[a] = type_eps[APR * t + s];
            gamma[a] = g_hydro * type_hydro[t];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Forward kinematics, eqs (kin_02)-(kin_04), (r1)                      */
/* ------------------------------------------------------------------ */
/* theta[j] holds the dihedral itself (phi or psi, radians).  The ZP value is pi,
 * so joint j turns by (theta[j] - pi) about its ZP axis u0_j (right-hand rule).
 * M_l = prod_{r<l} R(u0_r, theta_r - pi) orients link l (M_0 = I).  Body vectors
 * b_l = M_l b0_l chain the joint points; an atom of link l sits at
 * p_{l-1} + M_l (r0_a - p0_{l-1}).  Outputs: positions r, current joint axes u and
 * joint points p. */
int or_fk(int m, const double *r0, const double *theta, double *r, double *u, double *p)
{
    int n = APR * m, J = 2 * m, L = 2 * m + 1;
    double *M = (double *)malloc(sizeof(double) * 9 * L);
    double *u0 = (double *)malloc(sizeof(double) * 3 * J);
    double *p0 = (double *)malloc(sizeof(double) * 3 * J);
    double *pc = (double *)malloc(sizeof(double) * 3 * J);
    if (!M || !u0 || !p0 || !pc) { free(M); free(u0); free(p0); free(pc); return -2; }
    for (int j = 0; j < J; ++j) {
        int i = j / 2;
        const double *a = r0 + 3 * (APR * i + ((j % 2) ? A_CA : A_N));
        const double *b = r0 + 3 * (APR * i + ((j % 2) ? A_C : A_CA));
        double d[3];
        v_sub(b, a, d); v_unit(d, u0 + 3 * j);
        memcpy(p0 + 3 * j, a, sizeof(double) * 3);
    }
    /* sequential product of joint rotations (eq kin_04) */
    static const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    memcpy(M, I3, sizeof I3);
    for (int l = 1; l < L; ++l) {
        double Rj[9];
        m_rot(u0 + 3 * (l - 1), theta[l - 1] - OR_PI, Rj);
        m_mul(M + 9 * (l - 1), Rj, M + 9 * l);
    }
    /* joint points by the running sum of body vectors (eq r1); p_0 = N_0 is anchored */
    memcpy(pc, p0, sizeof(double) * 3);
    for (int j = 1; j < J; ++j) {
        double b0[3], b[3];
        v_sub(p0 + 3 * j, p0 + 3 * (j - 1), b0);
        m_vec(M + 9 * j, b0, b);       /* body vector between joints j-1 and j lies in link j */
        for (int k = 0; k < 3; ++k) pc[3 * j + k] = pc[3 * (j - 1) + k] + b[k];
    }
    for (int a = 0; a < n; ++a) {
        int l = or_link_of_atom(a);
        if (l == 0) { memcpy(r + 3 * a, r0 + 3 * a, sizeof(double) * 3); continue; }
        double d0[3], d[3];
        v_sub(r0 + 3 * a, p0 + 3 * (l - 1), d0);
        m_vec(M + 9 * l, d0, d);
        for (int k = 0; k < 3; ++k) r[3 * a + k] = pc[3 * (l - 1) + k] + d[k];
    }
    if (u) for (int j = 0; j < J; ++j) m_vec(M + 9 * (j + 1), u0 + 3 * j, u + 3 * j);
    if (p) memcpy(p, pc, sizeof(double) * 3 * J);
    free(M); free(u0); free(p0); free(pc);
    return 0;
}

/* The same kinematics one residue at a time, for preparing inputs (growing a
 * start conformation): given the rotation Mk of link 2k and the current point
 * pk of joint 2k (atom N of residue k), place the atoms of links 2k+1 and 2k+2
 * for angles (phi, psi) = (theta_2k, theta_2k+1): slots 2..9 of residue k and,
 * if k+1 < m, slots 0..1 of residue k+1, written to pos[10][3] in that order.
 * Returns in Mn, pn the rotation of link 2k+2 and the point of joint 2k+2.
 * Each value is computed by the operations of or_fk in the same order, so a
 * chain grown residue by residue equals or_fk of its angles. */
int or_fk_extend(int m, const double *r0, int k, const double *Mk, const double *pk, double phi, double psi,
                 double *pos, double *Mn, double *pn)
{
    if (k < 0 || k >= m) return -1;
    const double *N = r0 + 3 * (APR * k + A_N), *CA = r0 + 3 * (APR * k + A_CA), *Cc = r0 + 3 * (APR * k + A_C);
    double u0a[3], u0b[3], d[3];
    v_sub(CA, N, d); v_unit(d, u0a);   /* joint 2k: N -> CA, point N */
    v_sub(Cc, CA, d); v_unit(d, u0b);  /* joint 2k+1: CA -> C, point CA */
    double Ra[9], Rb[9], M1[9], M2[9];
    m_rot(u0a, phi - OR_PI, Ra);
    m_mul(Mk, Ra, M1);
    m_rot(u0b, psi - OR_PI, Rb);
    m_mul(M1, Rb, M2);
    double b0[3], b[3], p1[3];
    v_sub(CA, N, b0);
    m_vec(M1, b0, b);
    for (int q = 0; q < 3; ++q) p1[q] = pk[q] + b[q];
    int w = 0;
    for (int a = APR * k; a < APR * (k + 1) + 2 && a < APR * m; ++a) {
        const int l = or_link_of_atom(a);
        if (l != 2 * k + 1 && l != 2 * k + 2) continue;
        const double *M = l == 2 * k + 1 ? M1 : M2;
        const double *pc = l == 2 * k + 1 ? pk : p1;
        const double *p0 = l == 2 * k + 1 ? N : CA;
        double d0[3], dd[3];
        v_sub(r0 + 3 * a, p0, d0);
        m_vec(M, d0, dd);
        for (int q = 0; q < 3; ++q) pos[3 * w + q] = pc[q] + dd[q];
        ++w;
    }
    memcpy(Mn, M2, sizeof M2);
    if (k + 1 < m) {
        double c0[3], c[3];
        v_sub(r0 + 3 * (APR * (k + 1) + A_N), CA, c0);
        m_vec(M2, c0, c);
        for (int q = 0; q < 3; ++q) pn[q] = p1[q] + c[q];
    } else {
        memcpy(pn, p1, sizeof p1);
    }
    return w;
}

/* ------------------------------------------------------------------ */
/* Interaction classes by shortest bond path (Sec. 3.3)                 */
/* ------------------------------------------------------------------ */
/* Adjacency of the bond graph: up to 4 bonded partners per atom. */
static int *build_adjacency(int m)
{
    int n = APR * m, nb = or_bonds(m, NULL);
    int *bonds = (int *)malloc(sizeof(int) * 2 * nb);
    int *adj = (int *)malloc(sizeof(int) * 5 * n); /* [deg, p0, p1, p2, p3] */
    or_bonds(m, bonds);
    for (int a = 0; a < n; ++a) adj[5 * a] = 0;
    for (int e = 0; e < nb; ++e) {
        int x = bonds[2 * e], y = bonds[2 * e + 1];
        adj[5 * x + 1 + adj[5 * x]++] = y;
        adj[5 * y + 1 + adj[5 * y]++] = x;
    }
    free(bonds);
    return adj;
}

/* Bond-path length between atoms a and b, capped at 4 (4 = "four or more"):
 * breadth-first search from a over the bond graph, three levels deep. */
static int bond_path_adj(const int *adj, int a, int b)
{
    if (a == b) return 0;
    int seen[64], depth[64], ns = 0, head = 0;
    seen[ns] = a; depth[ns++] = 0;
    while (head < ns) {
        int x = seen[head], dx = depth[head++];
        if (dx == 3) continue;
        for (int t = 0; t < adj[5 * x]; ++t) {
            int y = adj[5 * x + 1 + t], dup = 0;
            for (int v = 0; v < ns; ++v) if (seen[v] == y) { dup = 1; break; }
            if (dup) continue;
            if (y == b) return dx + 1;
            seen[ns] = y; depth[ns++] = dx + 1;
        }
    }
    return 4;
}

int or_bond_path(int m, int a, int b)
{
    int *adj = build_adjacency(m);
    int d = bond_path_adj(adj, a, b);
    free(adj);
    return d;
}


/* ------------------------------------------------------------------ */
/* Coulomb + Lennard-Jones, eqs (02)-(03_9)                              */
/* ------------------------------------------------------------------ */
typedef struct {
    double cutoff, diel_k, w13, w14_elec, w14_vdw;
} or_pair_params;

/* Brute force over all pairs i<j with d <= cutoff (inclusive).  F[n][3] is
 * written; e_pair[2] = {E_elec, E_vdw}.  If subset != NULL only forces of the
 * listed atoms are computed (energies are then left zero). */
int or_pair_forces(int m, const double *r, const double *q, const double *R, const double *eps,
                   const or_pair_params *pp, const int *subset, int n_subset, double *F, double *e_pair)
{
    int n = APR * m;
    double Ee = 0.0, Ev = 0.0;
    int n_out = subset ? n_subset : n;
    int *adj = build_adjacency(m);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : Ee, Ev)
    for (int t = 0; t < n_out; ++t) {
        int i = subset ? subset[t] : t;
        double f[3] = {0, 0, 0};
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double dr[3];
            v_sub(r + 3 * i, r + 3 * j, dr);
            double d = v_norm(dr);
            if (!(d <= pp->cutoff)) continue;
            double we = 1.0, wv = 1.0;
            int path = (abs(i / APR - j / APR) > 1) ? 4 : bond_path_adj(adj, i, j);
            if (path <= 2) { we = (path == 1 ? 0.0 : pp->w13); wv = we; }
            else if (path == 3) { we = pp->w14_elec; wv = pp->w14_vdw; }
            if (we == 0.0 && wv == 0.0) continue;
            /* eq (02) with eps_ij = k_d d eps_0: E = C q_i q_j / (k_d d^2) */
            double Eel = we * OR_COULOMB * q[i] * q[j] / (pp->diel_k * d * d);
            double fel = 2.0 * Eel / d;                        /* -dE/dd */
            /* eq (03): E = eps_ij [(D/d)^12 - 2 (D/d)^6], D = R_i + R_j, eps_ij = sqrt(eps_i eps_j) */
            double D = R[i] + R[j], eij = sqrt(eps[i] * eps[j]);
            double s6 = pow(D / d, 6.0), s12 = s6 * s6;
            double Evw = wv * eij * (s12 - 2.0 * s6);
            double fvw = 12.0 * wv * eij * (s12 - s6) / d;     /* eq (03_1): 12 eps (D^12/d^13 - D^6/d^7) */
            double fm = (fel + fvw) / d;                       /* along e_ij = (r_i - r_j)/d */
            f[0] += fm * dr[0]; f[1] += fm * dr[1]; f[2] += fm * dr[2];
            if (!subset && j > i) { Ee += Eel; Ev += Evw; }
        }
        F[3 * i] = f[0]; F[3 * i + 1] = f[1]; F[3 * i + 2] = f[2];
    }
    if (e_pair) { e_pair[0] = subset ? 0.0 : Ee; e_pair[1] = subset ? 0.0 : Ev; }
    free(adj);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Offset-sphere samples (Sec. 3.4, polar geodesic sampling)            */
/* ------------------------------------------------------------------ */
/* n_orb orbits at polar angles t_o = pi (o + 1/2) / n_orb; orbit o carries
 * max(1, round(2 n_orb sin t_o)) points (proportional to its circumference),
 * evenly spaced in azimuth and offset by half a step on odd orbits.  Returns N
 * and writes Q[N][3] if Q != NULL. */
int or_samples(int n_orb, double *Q)
{
    int N = 0;
    for (int o = 0; o < n_orb; ++o) {
        double t = OR_PI * (o + 0.5) / n_orb;
        int no = (int)lround(2.0 * n_orb * sin(t));
        if (no < 1) no = 1;
        for (int k = 0; k < no; ++k) {
            double az = 2.0 * OR_PI * (k + 0.5 * (o % 2)) / no;
            if (Q) { Q[3 * N] = sin(t) * cos(az); Q[3 * N + 1] = sin(t) * sin(az); Q[3 * N + 2] = cos(t); }
            ++N;
        }
    }
    return N;
}

/* ------------------------------------------------------------------ */
/* Solvation energy and forces: Algorithm 1 with the C-state rules      */
/* ------------------------------------------------------------------ */
typedef struct {
    double delta_r;  /* finite difference (A) */
    double r_probe;  /* water probe radius (A) */
} or_sasa_params;

/* covered(q, c, Rad) per Sec. 3.4: ||q - c|| <= Rad.  Also tracks the smallest
 * |d^2 - Rad^2| seen, so a caller can tell whether a decision sat on a tie. */
static int covered(const double *qp, const double *c, double Rad, double *margin)
{
    double d[3];
    v_sub(qp, c, d);
    double e = v_dot(d, d) - Rad * Rad;
    double ae = fabs(e);
    if (margin && ae < *margin) *margin = ae;
    return e <= 0.0;
}

/* Neighbour lists: every j != i whose offset sphere, or its copy shifted by
 * delta_r, can reach a sample of atom i, i.e. d_ij <= Roff_i + Roff_j + delta_r.
 * Pairs beyond that bound change no count, so dropping them is exact (Sec. 2.2). */
static int *build_nbrs(int n, const double *r, const double *Roff, double dr, int **start_out)
{
    int *cnt = (int *)calloc(n + 1, sizeof(int));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int c = 0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            v_sub(r + 3 * i, r + 3 * j, d);
            double lim = Roff[i] + Roff[j] + dr;
            if (v_dot(d, d) <= lim * lim) ++c;
        }
        cnt[i + 1] = c;
    }
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    int *list = (int *)malloc(sizeof(int) * (cnt[n] > 0 ? cnt[n] : 1));
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        int c = cnt[i];
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            v_sub(r + 3 * i, r + 3 * j, d);
            double lim = Roff[i] + Roff[j] + dr;
            if (v_dot(d, d) <= lim * lim) list[c++] = j;
        }
    }
    *start_out = cnt;
    return list;
}

/* Algorithm 1.  Step 1 counts, per sample k of atom i, the neighbours whose
 * offset spheres cover it (C = 0, 1 or "2 or more") and remembers the single
 * overlapper when C = 1; the exposure ratio f_i drops by 1/N for every covered
 * sample and G_i = 4 pi gamma_i Roff_i^2 f_i (eq G_cav_patch).  Step 2 finds the
 * critical neighbours: for an exposed sample every neighbour j whose copy shifted
 * by delta_r e_s covers it (f_{i,j,s} falls by 1/N); for a critically overlapped
 * sample the one overlapper whose shifted copy no longer covers it (f_{i,j,s}
 * rises by 1/N).  Each event moves +-G0_i/(N delta_r) between F_i,s and F_j,s
 * with opposite signs (eqs F_cav_patch, finitediff).
 *
 * ev[i][slot][s] = N (f_{i,j,s} - f_i) for j = the slot-th neighbour of i.  The
 * force on atom i gathers its own sphere's events and its neighbours' events
 * in which i is the displaced atom, so no scatter is needed.
 *
 * Outputs: F[n][3]; f_exp[n] (optional); e_cav (total); margin (optional:
 * smallest |d^2 - R^2| over every coverage test made). */
int or_sasa_forces(int m, const double *r, const double *R, const double *gamma,
                   const double *Q, int N, const or_sasa_params *sp,
                   double *F, double *f_exp, double *e_cav, double *margin)
{
    int n = APR * m;
    double dr = sp->delta_r;
    double *Roff = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) Roff[i] = R[i] + sp->r_probe;
    int *nstart = NULL;
    int *nbr = build_nbrs(n, r, Roff, dr, &nstart);
    int total = nstart[n];
    int *ev = (int *)calloc((size_t)3 * (total > 0 ? total : 1), sizeof(int));
    double *G = (double *)malloc(sizeof(double) * n);
    double *fx = (double *)malloc(sizeof(double) * n);
    double min_margin = INFINITY;

#pragma omp parallel for schedule(dynamic, 8) reduction(min : min_margin)
    for (int i = 0; i < n; ++i) {
        double mg = INFINITY;
        int nn = nstart[i + 1] - nstart[i];
        const int *nb = nbr + nstart[i];
        int *evi = ev + 3 * nstart[i];
        int n_cov = 0;
        for (int k = 0; k < N; ++k) {
            double qp[3];
            for (int c = 0; c < 3; ++c) qp[c] = r[3 * i + c] + Roff[i] * Q[3 * k + c];
            /* Step 1 */
            int C = 0, jover = -1;
            for (int t = 0; t < nn && C < 2; ++t) {
                int j = nb[t];
                if (covered(qp, r + 3 * j, Roff[j], &mg)) {
                    ++C;
                    jover = (C == 1) ? t : -1;
                }
            }
            if (C >= 1) ++n_cov;
            /* Step 2 */
            for (int s = 0; s < 3; ++s) {
                if (C == 0) {
                    for (int t = 0; t < nn; ++t) {
                        double rj[3] = {r[3 * nb[t]], r[3 * nb[t] + 1], r[3 * nb[t] + 2]};
                        rj[s] += dr;
                        if (covered(qp, rj, Roff[nb[t]], &mg)) evi[3 * t + s] -= 1;
                    }
                } else if (C == 1) {
                    double rj[3] = {r[3 * nb[jover]], r[3 * nb[jover] + 1], r[3 * nb[jover] + 2]};
                    rj[s] += dr;
                    if (!covered(qp, rj, Roff[nb[jover]], &mg)) evi[3 * jover + s] += 1;
                }
            }
        }
        fx[i] = (double)(N - n_cov) / N;  /* exposed samples / N */
        G[i] = 4.0 * OR_PI * gamma[i] * Roff[i] * Roff[i];  /* G0_i */
        if (mg < min_margin) min_margin = mg;
    }

    double E = 0.0;
    for (int i = 0; i < n; ++i) E += G[i] * fx[i];
    if (f_exp) memcpy(f_exp, fx, sizeof(double) * n);

    /* eq (F_cav_patch): F_i,s = G0_i sum_j d_s f_i / dr (i's own sphere, j displaced)
     *                         - sum_j G0_j d_s f_j / dr (j's sphere, i displaced) */
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        double f[3] = {0, 0, 0};
        for (int t = nstart[i]; t < nstart[i + 1]; ++t) {
            int j = nbr[t];
            for (int s = 0; s < 3; ++s) f[s] += G[i] * ev[3 * t + s] / (N * dr);
            /* find i in j's list (lists are symmetric) */
            for (int u = nstart[j]; u < nstart[j + 1]; ++u) {
                if (nbr[u] != i) continue;
                for (int s = 0; s < 3; ++s) f[s] -= G[j] * ev[3 * u + s] / (N * dr);
                break;
            }
        }
        F[3 * i] = f[0]; F[3 * i + 1] = f[1]; F[3 * i + 2] = f[2];
    }
    if (e_cav) *e_cav = E;
    if (margin) *margin = min_margin;
    free(Roff); free(nstart); free(nbr); free(ev); free(G); free(fx);
    return 0;
}

/* Definitional form for tiny inputs (no C-state shortcut): f_{i,j,s} is
 * recounted from scratch with r_j replaced by r_j + delta_r e_s, for every
 * ordered pair (i, j != i) and axis s, and D[i][j][s] = N (f_{i,j,s} - f_i) is
 * returned as an integer.  O(n^3 N). */
int or_sasa_definitional(int m_or_n_atoms, int is_atoms, const double *r, const double *R,
                         const double *Q, int N, const or_sasa_params *sp, int *D, int *n_exposed)
{
    int n = is_atoms ? m_or_n_atoms : APR * m_or_n_atoms;
    double dr = sp->delta_r;
    double *Roff = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) Roff[i] = R[i] + sp->r_probe;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < n; ++i) {
        int base = 0;
        for (int k = 0; k < N; ++k) {
            double qp[3];
            for (int c = 0; c < 3; ++c) qp[c] = r[3 * i + c] + Roff[i] * Q[3 * k + c];
            int cov = 0;
            for (int j = 0; j < n; ++j) if (j != i && covered(qp, r + 3 * j, Roff[j], NULL)) { cov = 1; break; }
            if (!cov) ++base;
        }
        if (n_exposed) n_exposed[i] = base;
        for (int j = 0; j < n; ++j) {
            for (int s = 0; s < 3; ++s) {
                if (j == i) { D[((size_t)i * n + j) * 3 + s] = 0; continue; }
                int exp_count = 0;
                for (int k = 0; k < N; ++k) {
                    double qp[3];
                    for (int c = 0; c < 3; ++c) qp[c] = r[3 * i + c] + Roff[i] * Q[3 * k + c];
                    int cov = 0;
                    for (int jj = 0; jj < n && !cov; ++jj) {
                        if (jj == i) continue;
                        double c3[3] = {r[3 * jj], r[3 * jj + 1], r[3 * jj + 2]};
                        if (jj == j) c3[s] += dr;
                        if (covered(qp, c3, Roff[jj], NULL)) cov = 1;
                    }
                    if (!cov) ++exp_count;
                }
                D[((size_t)i * n + j) * 3 + s] = exp_count - base;
            }
        }
    }
    free(Roff);
    return 0;
}

/* The C-state event matrix on an arbitrary atom set (for comparison with the
 * definitional form): D[i][j][s] as above, from Algorithm 1's rules. */
int or_sasa_events(int n, const double *r, const double *R, const double *Q, int N,
                   const or_sasa_params *sp, int *D, int *n_exposed)
{
    double dr = sp->delta_r;
    double *Roff = (double *)malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) Roff[i] = R[i] + sp->r_probe;
    memset(D, 0, sizeof(int) * (size_t)n * n * 3);
    for (int i = 0; i < n; ++i) {
        int ex = 0;
        for (int k = 0; k < N; ++k) {
            double qp[3];
            for (int c = 0; c < 3; ++c) qp[c] = r[3 * i + c] + Roff[i] * Q[3 * k + c];
            int C = 0, jover = -1;
            for (int j = 0; j < n && C < 2; ++j) {
                if (j == i) continue;
                if (covered(qp, r + 3 * j, Roff[j], NULL)) { ++C; jover = (C == 1) ? j : -1; }
            }
            if (C == 0) ++ex;
            for (int s = 0; s < 3; ++s) {
                if (C == 0) {
                    for (int j = 0; j < n; ++j) {
                        if (j == i) continue;
                        double c3[3] = {r[3 * j], r[3 * j + 1], r[3 * j + 2]};
                        c3[s] += dr;
                        if (covered(qp, c3, Roff[j], NULL)) D[((size_t)i * n + j) * 3 + s] -= 1;
                    }
                } else if (C == 1) {
                    double c3[3] = {r[3 * jover], r[3 * jover + 1], r[3 * jover + 2]};
                    c3[s] += dr;
                    if (!covered(qp, c3, Roff[jover], NULL)) D[((size_t)i * n + jover) * 3 + s] += 1;
                }
            }
        }
        if (n_exposed) n_exposed[i] = ex;
    }
    free(Roff);
    return 0;
}

/* SASA forces/energy on an arbitrary atom set (not a chain): used by the
 * closed-form sphere checks.  Same rules as or_sasa_forces. */
int or_sasa_atoms(int n, const double *r, const double *R, const double *gamma, const double *Q, int N,
                  const or_sasa_params *sp, double *F, double *f_exp, double *e_cav)
{
    int *D = (int *)malloc(sizeof(int) * (size_t)n * n * 3);
    int *ex = (int *)malloc(sizeof(int) * n);
    or_sasa_events(n, r, R, Q, N, sp, D, ex);
    double E = 0.0;
    for (int i = 0; i < n; ++i) {
        double Ro = R[i] + sp->r_probe, G0 = 4.0 * OR_PI * gamma[i] * Ro * Ro;
        double fi = (double)ex[i] / N;
        if (f_exp) f_exp[i] = fi;
        E += G0 * fi;
    }
    for (int i = 0; i < n; ++i) {
        double Ri = R[i] + sp->r_probe, G0i = 4.0 * OR_PI * gamma[i] * Ri * Ri;
        double f[3] = {0, 0, 0};
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double Rj = R[j] + sp->r_probe, G0j = 4.0 * OR_PI * gamma[j] * Rj * Rj;
            for (int s = 0; s < 3; ++s)
                f[s] += (G0i * D[((size_t)i * n + j) * 3 + s] - G0j * D[((size_t)j * n + i) * 3 + s]) / (N * sp->delta_r);
        }
        for (int s = 0; s < 3; ++s) F[3 * i + s] = f[s];
    }
    if (e_cav) *e_cav = E;
    free(D); free(ex);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Side-chain joints (Sec. 2.1: chi dihedrals of the side-chain branch) */
/* ------------------------------------------------------------------ */
/* chi_i is the dihedral N-CA-CB-HB1 of residue i (60 degrees in the zero
 * position).  The branch it turns is HB1..HB3, which turn rigidly about the
 * CA->CB bond; nothing else moves.  Given the positions r of or_fk (the
 * branch at its zero-position chi), turn each residue's branch by
 * chi_i - 60 degrees about its current CA->CB axis (right-handed, so the
 * dihedral grows with chi) and return that axis and the point CA. */
int or_fk_chi(int m, const double *chi, double *r, double *u, double *p)
{
    for (int i = 0; i < m; ++i) {
        const double *CA = r + 3 * (APR * i + A_CA), *CB = r + 3 * (APR * i + A_CB);
        double d[3], ax[3], R[9];
        v_sub(CB, CA, d);
        v_unit(d, ax);
        m_rot(ax, chi[i] - deg(60.0), R);
        for (int h = A_HB1; h <= A_HB3; ++h) {
            double *x = r + 3 * (APR * i + h), e[3], f[3];
            v_sub(x, CB, e);
            m_vec(R, e, f);
            for (int k = 0; k < 3; ++k) x[k] = CB[k] + f[k];
        }
        if (u) memcpy(u + 3 * i, ax, sizeof ax);
        if (p) memcpy(p + 3 * i, CA, sizeof(double) * 3);
    }
    return 0;
}

/* tau_chi_i = u_i . sum over HB1..HB3 of residue i of (r_a - p_i) x F_a. */
int or_torques_chi(int m, const double *r, const double *F, const double *u, const double *p, double *tau)
{
    for (int i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int h = A_HB1; h <= A_HB3; ++h) {
            const int a = APR * i + h;
            double d[3], c[3];
            v_sub(r + 3 * a, p + 3 * i, d);
            v_cross(d, F + 3 * a, c);
            acc += v_dot(u + 3 * i, c);
        }
        tau[i] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Joint torques, eqs (KCM_01), (KCM_02), (KCM_04)-(KCM_06)             */
/* ------------------------------------------------------------------ */
/* Direct sum: tau_j = u_j . sum_{a in links > j} (r_a - p_j) x F_a. */
int or_torques(int m, const double *r, const double *F, const double *u, const double *p, double *tau)
{
    int n = APR * m, J = 2 * m;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < J; ++j) {
        double acc = 0.0;
        for (int a = 0; a < n; ++a) {
            if (or_link_of_atom(a) <= j) continue;
            double d[3], c[3];
            v_sub(r + 3 * a, p + 3 * j, d);
            v_cross(d, F + 3 * a, c);
            acc += v_dot(u + 3 * j, c);
        }
        tau[j] = acc;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Compliance step, eq (KCM_07), and the angle update of Sec. 3.1       */
/* ------------------------------------------------------------------ */
enum { OR_STEP_CAPPED = 0, OR_STEP_PAPER = 1, OR_STEP_LINEAR = 2 };

/* PAPER:  dtheta = s tau / |tau|_max            (eq KCM_07, s in rad)
 * LINEAR: dtheta = kappa tau
 * CAPPED: dtheta = kappa tau min(1, s / (kappa |tau|_max))
 * Masked joints (mask == 0) do not move and do not enter |tau|_max.  theta is
 * advanced and wrapped to (-pi, pi].  Returns max |dtheta| through *max_dtheta. */
int or_step(int J, const double *tau, const uint8_t *mask, int rule, double kappa, double s,
            double *theta, double *dtheta, double *max_dtheta)
{
    double tmax = 0.0;
    for (int j = 0; j < J; ++j)
        if (!mask || mask[j]) tmax = fmax(tmax, fabs(tau[j]));
    double scale;
    if (rule == OR_STEP_PAPER) scale = (tmax > 0.0) ? s / tmax : 0.0;
    else if (rule == OR_STEP_LINEAR) scale = kappa;
    else scale = (kappa * tmax > s) ? s / tmax : kappa;
    double mx = 0.0;
    for (int j = 0; j < J; ++j) {
        double d = (!mask || mask[j]) ? scale * tau[j] : 0.0;
        if (dtheta) dtheta[j] = d;
        mx = fmax(mx, fabs(d));
        double t = theta[j] + d;
        while (t > OR_PI) t -= 2.0 * OR_PI;
        while (t <= -OR_PI) t += 2.0 * OR_PI;
        theta[j] = t;
    }
    if (max_dtheta) *max_dtheta = mx;
    return 0;
}

/* The OpenMP thread count the oracle runs with. */
int or_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
