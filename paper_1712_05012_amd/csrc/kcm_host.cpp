// kcm_host.cpp -- host runtime of libkcm: chain construction, device block
// layout, batch tables, launch sequencing and the C ABI declared in kcm.h.
#include "../../include/kcm.h"
#include "kcm_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace kcm;

namespace {

// the calling thread's last error message, in a fixed buffer (setting it
// allocates nothing)
thread_local char g_err[512];

kcm_status fail(kcm_status s, const char *msg)
{
    std::snprintf(g_err, sizeof(g_err), "%s", msg);
    return s;
}
kcm_status fail(kcm_status s, const std::string &msg) { return fail(s, msg.c_str()); }

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(KCM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
    } while (0)

constexpr double kPi = 3.14159265358979323846;
constexpr double kCoulomb = 332.0636;  // kcal A / (mol e^2)

// ---------------------------------------------------------------------------
// residue template and zero position (Sec. 2.1)
// ---------------------------------------------------------------------------
struct V3 {
    double x, y, z;
};
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
V3 unit(V3 a) { return a * (1.0 / std::sqrt(dot(a, a))); }

// Atom d bonded to c with |cd| = len, angle b-c-d = ang, torsion a-b-c-d = tor (degrees).
V3 nerf(V3 a, V3 b, V3 c, double len, double ang, double tor)
{
    const V3 e1 = unit(c - b);
    const V3 nrm = unit(cross(b - a, e1));
    const V3 e2 = cross(nrm, e1);
    const double th = ang * kPi / 180.0, ph = tor * kPi / 180.0;
    return c + e1 * (-len * std::cos(th)) + e2 * (len * std::sin(th) * std::cos(ph)) + nrm * (len * std::sin(th) * std::sin(ph));
}

enum Slot { N_ = 0, H_, CA_, HA_, CB_, HB1_, HB2_, HB3_, C_, O_ };

// Ideal backbone (N-CA 1.458, CA-C 1.525, C-N 1.329 A; N-CA-C 111.2, CA-C-N 116.2,
// C-N-CA 121.7, CA-C=O 120.8 deg), tetrahedral CA and CB, amide H in plane.
// phi = psi = omega = 180 deg; N of residue 0 at the origin, CA on +x, C in the xy plane.
std::vector<V3> zero_position(int m)
{
    std::vector<V3> at(APR * m);
    auto A = [&](int i, int s) -> V3 & { return at[APR * i + s]; };
    const double ang_nh = 0.5 * (360.0 - 121.7);
    for (int i = 0; i < m; ++i) {
        if (i == 0) {
            A(0, N_) = {0.0, 0.0, 0.0};
            A(0, CA_) = {1.458, 0.0, 0.0};
            const double t = 111.2 * kPi / 180.0;
            A(0, C_) = {1.458 - 1.525 * std::cos(t), 1.525 * std::sin(t), 0.0};
        } else {
            A(i, N_) = nerf(A(i - 1, N_), A(i - 1, CA_), A(i - 1, C_), 1.329, 116.2, 180.0);
            A(i, CA_) = nerf(A(i - 1, CA_), A(i - 1, C_), A(i, N_), 1.458, 121.7, 180.0);
            A(i, C_) = nerf(A(i - 1, C_), A(i, N_), A(i, CA_), 1.525, 111.2, 180.0);
        }
        A(i, H_) = nerf(A(i, C_), A(i, CA_), A(i, N_), 1.01, ang_nh, 0.0);
        A(i, CB_) = nerf(A(i, C_), A(i, N_), A(i, CA_), 1.53, 109.5, -120.0);
        A(i, HA_) = nerf(A(i, C_), A(i, N_), A(i, CA_), 1.09, 109.5, 120.0);
        A(i, HB1_) = nerf(A(i, N_), A(i, CA_), A(i, CB_), 1.09, 109.5, 60.0);
        A(i, HB2_) = nerf(A(i, N_), A(i, CA_), A(i, CB_), 1.09, 109.5, 180.0);
        A(i, HB3_) = nerf(A(i, N_), A(i, CA_), A(i, CB_), 1.09, 109.5, -60.0);
        A(i, O_) = nerf(A(i, N_), A(i, CA_), A(i, C_), 1.231, 120.8, 0.0);
    }
    return at;
}

// Interaction classes by bond-path length (Sec. 3.3), as bitmasks per slot of
// the middle residue of a three-residue window: bit t marks window atom t
// (t = 10 (dres + 1) + slot).  Paths of length <= 3 never leave the window, so
// the same masks serve every residue of every chain.
void bond_class_masks(uint32_t m12[APR], uint32_t m13[APR], uint32_t m14[APR])
{
    const int W = 3 * APR;
    static const int intra[][2] = {{N_, H_},   {N_, CA_},  {CA_, HA_}, {CA_, CB_}, {CA_, C_},
                                   {CB_, HB1_}, {CB_, HB2_}, {CB_, HB3_}, {C_, O_}};
    std::vector<std::vector<int>> adj(W);
    for (int r = 0; r < 3; ++r) {
        for (auto &b : intra) {
            adj[APR * r + b[0]].push_back(APR * r + b[1]);
            adj[APR * r + b[1]].push_back(APR * r + b[0]);
        }
        if (r < 2) {
            adj[APR * r + C_].push_back(APR * (r + 1) + N_);
            adj[APR * (r + 1) + N_].push_back(APR * r + C_);
        }
    }
    for (int s = 0; s < APR; ++s) {
        std::vector<int> dist(W, -1), queue{APR + s};
        dist[APR + s] = 0;
        for (size_t h = 0; h < queue.size(); ++h)
            for (int y : adj[queue[h]])
                if (dist[y] < 0) {
                    dist[y] = dist[queue[h]] + 1;
                    queue.push_back(y);
                }
        m12[s] = m13[s] = m14[s] = 0;
        for (int t = 0; t < W; ++t) {
            if (dist[t] == 1) m12[s] |= 1u << t;
            if (dist[t] == 2) m13[s] |= 1u << t;
            if (dist[t] == 3) m14[s] |= 1u << t;
        }
    }
}

// The bond classes of each slot as one word (two bits per atom of the
// three-residue window), and the pair weights of each class in both
// precisions, taken exactly as the force kernel applies them: the term flag
// (1 or 0) times the class factor.
template <typename Real>
static int class_weights(const ChainDev &h, Real *tab)
{
    const Real we0 = (h.terms & KCM_TERM_ELEC) ? (Real)1 : (Real)0, wv0 = (h.terms & KCM_TERM_VDW) ? (Real)1 : (Real)0;
    int skip = 0;
    for (int c = 0; c < 4; ++c) {
        Real we = we0, wv = wv0;
        if (c == 1) { we = 0; wv = 0; }
        else if (c == 2) { we *= (Real)h.w13; wv *= (Real)h.w13; }
        else if (c == 3) { we *= (Real)h.w14e; wv *= (Real)h.w14v; }
        tab[2 * c] = we;
        tab[2 * c + 1] = wv;
        if (we == (Real)0 && wv == (Real)0) skip |= 1 << c;
    }
    return skip;
}

void bond_class_table(ChainDev &h)
{
    for (int s = 0; s < APR; ++s) {
        uint64_t w = 0;
        for (int t = 0; t < 3 * APR; ++t) {
            const uint32_t bit = 1u << t;
            const uint64_t c = (h.m12[s] & bit) ? 1 : (h.m13[s] & bit) ? 2 : (h.m14[s] & bit) ? 3 : 0;
            w |= c << (2 * t);
        }
        h.cls_word[s] = w;
    }
    h.skip_cls32 = class_weights<float>(h, h.wtab32);
    h.skip_cls64 = class_weights<double>(h, h.wtab64);
}

// Polar geodesic samples (Sec. 3.4): n_orb orbits at polar angles pi (o + 1/2) / n_orb,
// round(2 n_orb sin) points on each (at least one), evenly spaced in azimuth,
// odd orbits offset by half a step.
std::vector<V3> sample_directions(int n_orb)
{
    std::vector<V3> q;
    for (int o = 0; o < n_orb; ++o) {
        const double polar = kPi * (o + 0.5) / n_orb;
        const int cnt = std::max(1, (int)std::lround(2.0 * n_orb * std::sin(polar)));
        for (int p = 0; p < cnt; ++p) {
            const double az = 2.0 * kPi * (p + 0.5 * (o & 1)) / cnt;
            q.push_back({std::sin(polar) * std::cos(az), std::sin(polar) * std::sin(az), std::cos(polar)});
        }
    }
    return q;
}

// ---------------------------------------------------------------------------
// device block layout
// ---------------------------------------------------------------------------
struct Layout {
    size_t desc, stats, grid, theta, dtheta, tau, mc_theta, mask, joint0, jcur, xform, xform_loc, blk_xf, tmax_part, bad_part;
    size_t r0, r, aparam, g0, qfix;
    size_t cell_key, cell_count, cell_start, cell_local, scan_part, bbox_part, wrench_part, s_r, s_p, s_tmp, s_idx;
    size_t f_pair, f_cav;
    size_t e_atom;
    size_t q64, q32;
    size_t total;
    int n, J, L, N, cap;
    int n_chi, Jt, njb_bb, njb;  // side-chain joints, all joints, backbone and all joint blocks
};

static_assert((8LL * APR * (1 << 19) + SCAN_CHUNK - 1) / SCAN_CHUNK <= SCAN_MAX_CHUNKS,
              "the largest chain's grid capacity must fit the scan's chunk table");

Layout make_layout(int m, int n_orb, int side_chains)
{
    Layout l{};
    l.n = APR * m;
    l.J = 2 * m;
    l.L = 2 * m + 1;
    l.n_chi = side_chains ? m : 0;
    l.Jt = l.J + l.n_chi;
    l.njb_bb = (l.J + JOINT_BLOCK - 1) / JOINT_BLOCK;
    l.njb = l.njb_bb + (l.n_chi + JOINT_BLOCK - 1) / JOINT_BLOCK;
    l.N = (int)sample_directions(n_orb).size();
    l.cap = std::max(8192, 8 * l.n);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        const size_t o = off;
        off += bytes;
        return o;
    };
    const size_t n = l.n, J = l.J, L = l.L, N = l.N, cap = l.cap;
    l.desc = take(sizeof(ChainDev));
    l.stats = take(sizeof(ChainStats));
    l.grid = take(sizeof(Grid));
    const size_t Jt = l.Jt;
    l.theta = take(8 * Jt);
    l.dtheta = take(8 * Jt);
    l.tau = take(8 * Jt);
    l.mc_theta = take(16 * Jt);
    l.mask = take(Jt);
    l.joint0 = take(64 * J);
    l.jcur = take(64 * J);
    l.xform = take(96 * L);
    l.xform_loc = take(96 * J);
    l.blk_xf = take(96 * (size_t)l.njb_bb);
    l.tmax_part = take(8 * (size_t)l.njb);
    l.bad_part = take(4 * (size_t)l.njb);
    l.r0 = take(32 * n);
    l.r = take(32 * n);
    l.aparam = take(32 * n);
    l.g0 = take(8 * n);
    l.qfix = take(8 * n);
    l.cell_key = take(4 * n);
    l.cell_count = take(4 * cap);
    l.cell_start = take(4 * (cap + 1));
    l.cell_local = take(4 * cap);
    l.scan_part = take(4 * ((cap + SCAN_CHUNK - 1) / SCAN_CHUNK));
    const size_t nblk = (n + ATOM_BLOCK - 1) / ATOM_BLOCK;
    l.bbox_part = take(8 * 6 * nblk);
    l.wrench_part = take(8 * WPART * nblk);
    l.s_r = take(32 * n);
    l.s_p = take(32 * n);
    l.s_tmp = take(4 * n);
    l.s_idx = take(4 * n);
    l.f_pair = take(32 * n);
    l.f_cav = take(24 * n);
    l.e_atom = take(32 * n);
    l.q64 = take(32 * N);
    l.q32 = take(16 * N);
    l.total = (off + 255) & ~size_t(255);
    return l;
}

kcm_status check_inputs(const kcm_chain_desc *d, const kcm_params *p)
{
    if (!d || !p) return fail(KCM_E_INVAL, "null desc or params");
    // the grid capacity (8 cells per atom) must fit the scan's chunk table
    if (d->n_res < 1 || d->n_res > (1 << 19)) return fail(KCM_E_INVAL, "n_res out of range (1 .. 524288)");
    if (d->side_chains != 0 && d->side_chains != 1) return fail(KCM_E_INVAL, "side_chains must be 0 or 1");
    if (!d->res_type || !d->types || d->n_types < 1) return fail(KCM_E_INVAL, "missing residue types");
    for (int i = 0; i < d->n_res; ++i)
        if (d->res_type[i] < 0 || d->res_type[i] >= d->n_types) return fail(KCM_E_INVAL, "res_type out of range");
    if (!(p->cutoff > 0.0) || !(p->delta_r > 0.0) || !(p->r_probe >= 0.0) || !(p->kappa >= 0.0) || !(p->max_step > 0.0))
        return fail(KCM_E_INVAL, "cutoff, delta_r, r_probe, kappa or max_step out of range");
    if (p->n_orbits < 1 || p->n_orbits > 64) return fail(KCM_E_INVAL, "n_orbits must be in 1..64");
    if ((int)sample_directions(p->n_orbits).size() > 32767) return fail(KCM_E_INVAL, "too many samples");
    if (p->step_rule < 0 || p->step_rule > 2) return fail(KCM_E_INVAL, "bad step_rule");
    if (p->precision != KCM_FP64 && p->precision != KCM_MIXED) return fail(KCM_E_INVAL, "bad precision");
    if (p->terms < 0 || p->terms > KCM_TERM_ALL) return fail(KCM_E_INVAL, "bad terms");
    if (!(p->diel_k > 0.0)) return fail(KCM_E_INVAL, "diel_k must be > 0");
    if (!(p->cell_size >= 0.0)) return fail(KCM_E_INVAL, "cell_size must be >= 0");
    return KCM_OK;
}

// ---------------------------------------------------------------------------
// batch tables: per (device, stream) a device array of chain descriptors and
// the cumulative atom offsets the force kernel maps its workgroups with
// ---------------------------------------------------------------------------
struct Table {
    int device = -1;
    hipStream_t stream = nullptr;
    std::vector<const kcm_chain *> chains;
    void *dev = nullptr;
    size_t cap = 0;
    Batch batch{};
    hipGraphExec_t graph = nullptr;  // one iteration, captured for this batch
    int graph_prec = -1;
    hipGraphExec_t graph_n = nullptr;  // graph_n_depth iterations in one graph
    int graph_n_prec = -1, graph_n_depth = 0;
    ChainStats *stats_dev = nullptr;   // [stats_cap] the batch's records, gathered on the device
    ChainStats *stats_host = nullptr;  // [stats_cap] pinned host copy of them
    int stats_cap = 0;
    int64_t *mc_off_dev = nullptr;     // [mc_off_cap] per-chain offsets into a Monte Carlo call's perturbations
    int mc_off_cap = 0;
};

std::mutex g_mu;
std::vector<Table> g_tables;
int g_graphs = 1;                       // iterations per captured graph (0: direct launches)
int g_force_shape = 0;                  // launch shape of the force kernel (kcm_set_force_variant)
constexpr int kMaxGraphDepth = 64;
std::vector<std::pair<int, hipStream_t>> g_capture_streams;  // per device

hipError_t capture_stream(hipStream_t *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    for (auto &p : g_capture_streams)
        if (p.first == dev) {
            *out = p.second;
            return hipSuccess;
        }
    hipStream_t s = nullptr;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    g_capture_streams.emplace_back(dev, s);
    *out = s;
    return hipSuccess;
}

struct TimedIter {
    hipEvent_t it0, f0, f1, it1;
};

// One iteration; with ti, events bracket the iteration and the force kernel.
hipError_t launch_iteration(const Batch &bt, int prec, hipStream_t stream, const TimedIter *ti = nullptr)
{
    hipError_t e;
    if (ti && (e = hipEventRecord(ti->it0, stream)) != hipSuccess) return e;
    if ((e = launch_tau(bt, stream)) != hipSuccess) return e;
    if ((e = launch_stepfk(bt, MODE_ITER, stream)) != hipSuccess) return e;
    if ((e = launch_place(bt, MODE_ITER, stream)) != hipSuccess) return e;
    if ((e = launch_cellkey(bt, stream)) != hipSuccess) return e;
    if ((e = launch_cellscan(bt, stream)) != hipSuccess) return e;
    if ((e = launch_scatter(bt, stream)) != hipSuccess) return e;
    if ((e = launch_rank(bt, stream)) != hipSuccess) return e;
    if (ti && (e = hipEventRecord(ti->f0, stream)) != hipSuccess) return e;
    if ((e = launch_force(bt, prec, g_force_shape, stream)) != hipSuccess) return e;
    if (ti && (e = hipEventRecord(ti->f1, stream)) != hipSuccess) return e;
    if ((e = launch_wrench(bt, stream)) != hipSuccess) return e;
    if (ti && (e = hipEventRecord(ti->it1, stream)) != hipSuccess) return e;
    return hipSuccess;
}

// Positions and the first grid of every chain of the batch that has none
// (the kernels skip the others).
hipError_t launch_boot(const Batch &bt, hipStream_t stream)
{
    hipError_t e;
    if ((e = launch_stepfk(bt, MODE_BOOT, stream)) != hipSuccess) return e;
    if ((e = launch_place(bt, MODE_BOOT, stream)) != hipSuccess) return e;
    return launch_gridboot(bt, stream);
}

// The post phase of the last forces of a call.
hipError_t launch_final(const Batch &bt, hipStream_t stream)
{
    hipError_t e;
    if ((e = launch_tau(bt, stream)) != hipSuccess) return e;
    if ((e = launch_stepfk(bt, MODE_FINAL, stream)) != hipSuccess) return e;
    return launch_finish(bt, stream);
}

// Captures `iters` consecutive iterations of the batch as one executable graph.
hipError_t capture_iterations(const Batch &bt, int prec, int iters, hipGraphExec_t *out)
{
    hipStream_t cs = nullptr;
    hipError_t e = capture_stream(&cs);
    if (e != hipSuccess) return e;
    hipGraph_t g = nullptr;
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    hipError_t le = hipSuccess;
    for (int i = 0; i < iters && le == hipSuccess; ++i) le = launch_iteration(bt, prec, cs);
    hipError_t ee = hipStreamEndCapture(cs, &g);
    if (le != hipSuccess) return le;
    if (ee != hipSuccess) return ee;
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipError_t de = hipGraphDestroy(g);
    if (e != hipSuccess) {
        *out = nullptr;
        return e;
    }
    return de;
}
std::vector<TimedIter> g_timed;
std::vector<hipEvent_t> g_event_pool;
int g_timing = 0;
int64_t g_timing_count = 0;
double g_force_ms = 0.0, g_iter_ms = 0.0;
int64_t g_force_n = 0, g_iter_n = 0;

hipEvent_t pooled_event()
{
    if (!g_event_pool.empty()) {
        hipEvent_t e = g_event_pool.back();
        g_event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

}  // namespace

struct kcm_chain {
    ChainDev h;          // host copy of the device descriptor
    ChainDev *d_desc;    // where it lives on the device
    void *dev_mem;
    size_t bytes;
    int device;
    int m, n, J, N;      // J: all joints (backbone, then side chains)
    int njb;             // joint blocks (backbone blocks, then side-chain blocks)
    std::vector<unsigned char> staging;  // host source of the build copies
    bool boot = true;    // the conformation has no grid yet (built, or new angles)
};

namespace {

kcm_status ensure_table(kcm_chain *const *chains, int n_chains, hipStream_t stream, Table **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    Table *t = nullptr;
    for (auto &x : g_tables)
        if (x.device == dev && x.stream == stream) t = &x;
    if (!t) {
        g_tables.emplace_back();
        t = &g_tables.back();
        t->device = dev;
        t->stream = stream;
    }
    bool same = (int)t->chains.size() == n_chains;
    for (int i = 0; same && i < n_chains; ++i) same = t->chains[i] == chains[i];
    if (!same) {
        const size_t ints = ((sizeof(int32_t) * (n_chains + 1) + 255) & ~size_t(255));
        const size_t off_pos = (sizeof(ChainDev *) * n_chains + 255) & ~size_t(255);
        const size_t blk_pos = off_pos + ints;
        const size_t jblk_pos = blk_pos + ints;
        const size_t scan_pos = jblk_pos + ints;
        const size_t need = scan_pos + sizeof(int32_t) * (n_chains + 1);
        if (need > t->cap) {
            if (t->dev) {
                HIP_TRY(hipStreamSynchronize(stream));
                HIP_TRY(hipFree(t->dev));
                t->dev = nullptr;
            }
            const size_t cap = std::max(need * 2, size_t(4096));
            HIP_TRY(hipMalloc(&t->dev, cap));
            t->cap = cap;
        }
        std::vector<unsigned char> host(need);
        ChainDev **tab = reinterpret_cast<ChainDev **>(host.data());
        int32_t *off = reinterpret_cast<int32_t *>(host.data() + off_pos);
        int32_t *blk = reinterpret_cast<int32_t *>(host.data() + blk_pos);
        int32_t *jblk = reinterpret_cast<int32_t *>(host.data() + jblk_pos);
        int32_t *sblk = reinterpret_cast<int32_t *>(host.data() + scan_pos);
        long long total = 0, blocks = 0, jblocks = 0, sblocks = 0;
        int max_chunks = 1;
        for (int i = 0; i < n_chains; ++i) {
            tab[i] = chains[i]->d_desc;
            off[i] = (int32_t)total;
            blk[i] = (int32_t)blocks;
            jblk[i] = (int32_t)jblocks;
            sblk[i] = (int32_t)sblocks;
            total += chains[i]->n;
            blocks += (chains[i]->n + ATOM_BLOCK - 1) / ATOM_BLOCK;
            jblocks += chains[i]->njb;
            const int chunks = (chains[i]->h.cap_cells + SCAN_CHUNK - 1) / SCAN_CHUNK;
            sblocks += chunks;
            max_chunks = std::max(max_chunks, chunks);
        }
        if (total > std::numeric_limits<int32_t>::max() || sblocks > std::numeric_limits<int32_t>::max())
            return fail(KCM_E_INVAL, "too many atoms in one call");
        off[n_chains] = (int32_t)total;
        blk[n_chains] = (int32_t)blocks;
        jblk[n_chains] = (int32_t)jblocks;
        sblk[n_chains] = (int32_t)sblocks;
        HIP_TRY(hipMemcpyAsync(t->dev, host.data(), need, hipMemcpyHostToDevice, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        unsigned char *d = static_cast<unsigned char *>(t->dev);
        t->batch.table = reinterpret_cast<ChainDev *const *>(d);
        t->batch.atom_off = reinterpret_cast<const int32_t *>(d + off_pos);
        t->batch.blk_off = reinterpret_cast<const int32_t *>(d + blk_pos);
        t->batch.jblk_off = reinterpret_cast<const int32_t *>(d + jblk_pos);
        t->batch.scan_off = reinterpret_cast<const int32_t *>(d + scan_pos);
        t->batch.n_chains = n_chains;
        t->batch.total_atoms = (int)total;
        t->batch.total_blocks = (int)blocks;
        t->batch.total_jblocks = (int)jblocks;
        t->batch.total_scan_blocks = (int)sblocks;
        t->batch.max_scan_chunks = max_chunks;
        t->chains.assign(chains, chains + n_chains);
        if (t->graph) {
            HIP_TRY(hipGraphExecDestroy(t->graph));
            t->graph = nullptr;
        }
        if (t->graph_n) {
            HIP_TRY(hipGraphExecDestroy(t->graph_n));
            t->graph_n = nullptr;
        }
    }
    *out = t;
    return KCM_OK;
}

template <typename T>
kcm_status write_field(T *dev_field, T value, hipStream_t s)
{
    HIP_TRY(hipMemcpyAsync(dev_field, &value, sizeof(T), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return KCM_OK;
}

// The records of every chain of the table's batch, read back with one gather
// kernel and one copy.  Synchronises the stream.
kcm_status gather_stats(Table *t, hipStream_t stream, std::vector<ChainStats> &out)
{
    const int n = t->batch.n_chains;
    if (n > t->stats_cap) {
        HIP_TRY(hipStreamSynchronize(stream));
        if (t->stats_dev) HIP_TRY(hipFree(t->stats_dev));
        if (t->stats_host) HIP_TRY(hipHostFree(t->stats_host));
        t->stats_dev = nullptr;
        t->stats_host = nullptr;
        t->stats_cap = 0;
        const int cap = std::max(2 * n, 64);
        HIP_TRY(hipMalloc(&t->stats_dev, sizeof(ChainStats) * cap));
        HIP_TRY(hipHostMalloc(&t->stats_host, sizeof(ChainStats) * cap, hipHostMallocDefault));
        t->stats_cap = cap;
    }
    HIP_TRY(launch_stats_gather(t->batch, t->stats_dev, stream));
    HIP_TRY(hipMemcpyAsync(t->stats_host, t->stats_dev, sizeof(ChainStats) * n, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    out.assign(t->stats_host, t->stats_host + n);
    return KCM_OK;
}

// Whether kernels may read p: device, managed or pinned host memory known to
// HIP.  Pageable host memory (or an unknown address) is not.
bool device_readable(const void *p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged || a.type == hipMemoryTypeHost;
}

// Device offsets of per-chain blocks of `per_joint` x J_c doubles laid one
// after the other in call order, in the table's offset buffer.  Synchronises.
kcm_status upload_joint_offsets(Table *t, kcm_chain *const *chains, int n_chains, int64_t per_joint,
                                hipStream_t stream)
{
    if (n_chains + 1 > t->mc_off_cap) {
        HIP_TRY(hipStreamSynchronize(stream));
        if (t->mc_off_dev) HIP_TRY(hipFree(t->mc_off_dev));
        t->mc_off_dev = nullptr;
        t->mc_off_cap = 0;
        const int cap = std::max(2 * (n_chains + 1), 64);
        HIP_TRY(hipMalloc(&t->mc_off_dev, sizeof(int64_t) * cap));
        t->mc_off_cap = cap;
    }
    std::vector<int64_t> off(n_chains + 1, 0);
    for (int i = 0; i < n_chains; ++i) off[i + 1] = off[i] + per_joint * chains[i]->J;
    HIP_TRY(hipMemcpyAsync(t->mc_off_dev, off.data(), sizeof(int64_t) * (n_chains + 1), hipMemcpyHostToDevice,
                           stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return KCM_OK;
}

kcm_status check_chains(kcm_chain *const *chains, int n_chains, int *precision)
{
    if (!chains || n_chains < 1) return fail(KCM_E_INVAL, "no chains");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    for (int i = 0; i < n_chains; ++i) {
        if (!chains[i]) return fail(KCM_E_INVAL, "null chain handle");
        if (chains[i]->device != dev) return fail(KCM_E_INVAL, "chain lives on another device");
        if (chains[i]->h.precision != chains[0]->h.precision) return fail(KCM_E_INVAL, "chains of one call must share precision");
    }
    std::vector<const kcm_chain *> sorted(chains, chains + n_chains);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end())
        return fail(KCM_E_INVAL, "a chain appears twice in one call");
    *precision = chains[0]->h.precision;
    return KCM_OK;
}

}  // namespace

extern "C" {

void kcm_default_params(kcm_params *p)
{
    if (!p) return;
    p->cutoff = 10.0;
    p->kappa = 1e-3;
    p->max_step = 1e-3;
    p->step_rule = KCM_STEP_CAPPED;
    p->precision = KCM_FP64;
    p->terms = KCM_TERM_ALL;
    p->n_orbits = 14;
    p->diel_k = 4.0;
    p->w13 = 0.0;
    p->w14_elec = 1.0 / 1.2;
    p->w14_vdw = 0.5;
    p->delta_r = 0.05;
    p->r_probe = 1.4;
    p->g_hydro = 0.025;
    p->cell_size = 0.0;
}

const char *kcm_last_error(void) { return g_err; }

kcm_status kcm_chain_bytes(const kcm_chain_desc *desc, const kcm_params *params, size_t *bytes)
{
    if (!bytes) return fail(KCM_E_INVAL, "null bytes");
    kcm_status s = check_inputs(desc, params);
    if (s != KCM_OK) return s;
    *bytes = make_layout(desc->n_res, params->n_orbits, desc->side_chains).total;
    return KCM_OK;
}

kcm_status kcm_build_chain(const kcm_chain_desc *desc, const kcm_params *params, void *dev_mem, size_t bytes,
                           void *hip_stream, kcm_chain **out)
{
    if (!out) return fail(KCM_E_INVAL, "null out");
    *out = nullptr;
    kcm_status s = check_inputs(desc, params);
    if (s != KCM_OK) return s;
    if (!dev_mem || (reinterpret_cast<uintptr_t>(dev_mem) & 255)) return fail(KCM_E_INVAL, "dev_mem must be 256-byte aligned");
    const int m = desc->n_res;
    const Layout l = make_layout(m, params->n_orbits, desc->side_chains);
    if (bytes < l.total) return fail(KCM_E_NOMEM, "device block smaller than kcm_chain_bytes");
    if (!device_readable(dev_mem)) return fail(KCM_E_INVAL, "dev_mem must be device memory");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);

    kcm_chain *c = new kcm_chain();
    c->dev_mem = dev_mem;
    c->bytes = bytes;
    c->m = m;
    c->n = l.n;
    c->J = l.Jt;
    c->njb = l.njb;
    c->N = l.N;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    unsigned char *base = static_cast<unsigned char *>(dev_mem);

    ChainDev &h = c->h;
    std::memset(&h, 0, sizeof h);
    h.n_atoms = l.n;
    h.n_joints = l.J;
    h.n_chi = l.n_chi;
    h.n_bb_blocks = l.njb_bb;
    h.n_links = l.L;
    h.n_samples = l.N;
    h.cap_cells = l.cap;
    h.precision = params->precision;
    h.terms = params->terms;
    h.step_rule = params->step_rule;
    h.cutoff = params->cutoff;
    h.kappa = params->kappa;
    h.max_step = params->max_step;
    h.diel_k = params->diel_k;
    h.coulomb = kCoulomb / params->diel_k;
    h.w13 = params->w13;
    h.w14e = params->w14_elec;
    h.w14v = params->w14_vdw;
    h.delta_r = params->delta_r;
    h.r_probe = params->r_probe;
    bond_class_masks(h.m12, h.m13, h.m14);
    bond_class_table(h);

    // per-atom inputs
    const double k6 = std::pow(2.0, 1.0 / 6.0);
    std::vector<double4> r0(l.n), apar(l.n);
    std::vector<double> g0(l.n);
    std::vector<long long> qfix(l.n);
    const std::vector<V3> zp = zero_position(m);
    double roff_max = 0.0;
    for (int a = 0; a < l.n; ++a) {
        const int i = a / APR, sl = a % APR;
        const kcm_residue_type &t = desc->types[desc->res_type[i]];
        const double R = 0.5 * k6 * t.sigma[sl];
        const double roff = R + params->r_probe;
        r0[a] = make_double4(zp[a].x, zp[a].y, zp[a].z, 0.0);
        apar[a] = make_double4(t.q[sl], R, std::sqrt(t.eps[sl]), roff);
        const double gamma = params->g_hydro * t.hydrophobicity;
        g0[a] = 4.0 * kPi * gamma * roff * roff;
        qfix[a] = std::llrint(g0[a] / (l.N * params->delta_r) * FIX_SCALE);
        roff_max = std::max(roff_max, roff);
        if (!(t.sigma[sl] > 0.0) || !(t.eps[sl] >= 0.0) || !std::isfinite(t.q[sl]) || !std::isfinite(t.hydrophobicity)) {
            delete c;
            return fail(KCM_E_INVAL, "residue-type parameters out of range");
        }
    }
    h.roff_max = roff_max;
    const double reach_len = std::max(params->cutoff, 2.0 * roff_max + params->delta_r) + 1e-7;
    h.cell_min = params->cell_size > 0.0 ? params->cell_size : 0.5 * reach_len;

    // joints: zero-position axis u0 and point p0 (phi_i: N_i -> CA_i; psi_i: CA_i -> C_i)
    std::vector<double4> joint0(2 * l.J);
    for (int j = 0; j < l.J; ++j) {
        const int i = j / 2;
        const V3 a = zp[APR * i + (j % 2 ? CA_ : N_)], b = zp[APR * i + (j % 2 ? C_ : CA_)];
        const V3 u = unit(b - a);
        joint0[2 * j] = make_double4(u.x, u.y, u.z, 0.0);
        joint0[2 * j + 1] = make_double4(a.x, a.y, a.z, 0.0);
    }
    std::vector<double> theta(l.Jt);
    std::vector<uint8_t> mask(l.Jt);
    for (int j = 0; j < l.Jt; ++j) {
        // zero position: phi = psi = 180 degrees, chi (N-CA-CB-HB1) = 60 degrees
        double t = desc->theta0 ? desc->theta0[j] : (j < l.J ? kPi : kPi / 3.0);
        if (!std::isfinite(t)) {
            delete c;
            return fail(KCM_E_INVAL, "theta0 not finite");
        }
        t = std::remainder(t, 2.0 * kPi);
        if (t <= -kPi) t += 2.0 * kPi;
        theta[j] = t;
        mask[j] = desc->joint_mask ? (desc->joint_mask[j] ? 1 : 0) : 1;
    }
    const std::vector<V3> qd = sample_directions(params->n_orbits);
    std::vector<double4> q64(l.N);
    std::vector<float4> q32(l.N);
    for (int k = 0; k < l.N; ++k) {
        q64[k] = make_double4(qd[k].x, qd[k].y, qd[k].z, 0.0);
        q32[k] = make_float4((float)qd[k].x, (float)qd[k].y, (float)qd[k].z, 0.0f);
    }
    ChainStats st{};
    st.tol = 0.0;
    st.iter_limit = std::numeric_limits<int64_t>::max();
    st.active = 1;
    st.run = 1;
    st.need_grid = 1;

#define PTR(field, type) h.field = reinterpret_cast<type>(base + l.field)
    PTR(theta, double *);
    PTR(dtheta, double *);
    PTR(tau, double *);
    PTR(mc_theta, double *);
    PTR(mask, uint8_t *);
    PTR(joint0, double4 *);
    PTR(jcur, double4 *);
    PTR(xform, double *);
    PTR(xform_loc, double *);
    PTR(blk_xf, double *);
    PTR(tmax_part, double *);
    PTR(bad_part, int32_t *);
    PTR(r0, double4 *);
    PTR(r, double4 *);
    PTR(aparam, double4 *);
    PTR(g0, double *);
    PTR(qfix, long long *);
    PTR(cell_key, int32_t *);
    PTR(cell_count, int32_t *);
    PTR(cell_start, int32_t *);
    PTR(cell_local, int32_t *);
    PTR(scan_part, int32_t *);
    PTR(bbox_part, double *);
    PTR(wrench_part, double *);
    PTR(s_r, double4 *);
    PTR(s_p, double4 *);
    PTR(s_tmp, int32_t *);
    PTR(s_idx, int32_t *);
    PTR(f_pair, double4 *);
    PTR(f_cav, long long *);
    PTR(e_atom, double4 *);
    PTR(q64, double4 *);
    PTR(q32, float4 *);
    PTR(grid, Grid *);
    PTR(stats, ChainStats *);
#undef PTR
    c->d_desc = reinterpret_cast<ChainDev *>(base + l.desc);

    // one host staging image of every initialised region, copied in one go
    const size_t img = l.q32 + 16 * (size_t)l.N;
    c->staging.assign(img, 0);
    auto put = [&](size_t off, const void *src, size_t nbytes) { std::memcpy(c->staging.data() + off, src, nbytes); };
    put(l.desc, &h, sizeof h);
    put(l.stats, &st, sizeof st);
    put(l.theta, theta.data(), 8 * (size_t)l.Jt);
    put(l.mask, mask.data(), (size_t)l.Jt);
    put(l.joint0, joint0.data(), 32 * joint0.size());
    put(l.r0, r0.data(), 32 * (size_t)l.n);
    put(l.aparam, apar.data(), 32 * (size_t)l.n);
    put(l.g0, g0.data(), 8 * (size_t)l.n);
    put(l.qfix, qfix.data(), 8 * (size_t)l.n);
    put(l.q64, q64.data(), 32 * (size_t)l.N);
    put(l.q32, q32.data(), 16 * (size_t)l.N);
    hipError_t e = hipMemsetAsync(dev_mem, 0, l.total, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(dev_mem, c->staging.data(), img, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        delete c;
        return fail(KCM_E_DEVICE, std::string("build copy: ") + hipGetErrorString(e));
    }
    *out = c;
    return KCM_OK;
}

kcm_status kcm_chain_info(const kcm_chain *c, int32_t *n_atoms, int32_t *n_joints, int32_t *n_samples, int32_t *precision)
{
    if (!c) return fail(KCM_E_INVAL, "null chain");
    if (n_atoms) *n_atoms = c->n;
    if (n_joints) *n_joints = c->J;
    if (n_samples) *n_samples = c->N;
    if (precision) *precision = c->h.precision;
    return KCM_OK;
}

namespace {

// n_iter iterations of the table's batch (HIP graphs where captured); boot
// sequence first when a chain needs one or boot_all is set; the post phase of
// the last forces only when final is set
kcm_status iterate_locked(Table *t, kcm_chain *const *chains, int n_chains, int n_iter, int prec, hipStream_t stream,
                          bool boot_all, bool final)
{
    const Batch &bt = t->batch;
    const int depth = g_graphs;
    // a captured graph holds the precision's kernels in the current force shape
    const int key = prec + 16 * g_force_shape;
    if (depth > 0 && n_iter > 0 && (!t->graph || t->graph_prec != key)) {
        if (t->graph) {
            HIP_TRY(hipGraphExecDestroy(t->graph));
            t->graph = nullptr;
        }
        hipError_t e = capture_iterations(bt, prec, 1, &t->graph);
        if (e != hipSuccess) return fail(KCM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        t->graph_prec = key;
    }
    if (depth > 1 && n_iter >= depth && (!t->graph_n || t->graph_n_prec != key || t->graph_n_depth != depth)) {
        if (t->graph_n) {
            HIP_TRY(hipGraphExecDestroy(t->graph_n));
            t->graph_n = nullptr;
        }
        hipError_t e = capture_iterations(bt, prec, depth, &t->graph_n);
        if (e != hipSuccess) return fail(KCM_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        t->graph_n_prec = key;
        t->graph_n_depth = depth;
    }
    if (n_iter > 0) {
        bool boot = boot_all;
        for (int i = 0; i < n_chains; ++i) boot = boot || chains[i]->boot;
        if (boot) {
            HIP_TRY(launch_boot(bt, stream));
            for (int i = 0; i < n_chains; ++i) chains[i]->boot = false;
        }
    }
    for (int it = 0; it < n_iter;) {
        const bool timed = g_timing > 0 && (g_timing_count % g_timing) == 0;
        if (!timed) {
            // iterations until the next sampled one (or the end of the call)
            int run = n_iter - it;
            if (g_timing > 0) run = std::min<int64_t>(run, g_timing - g_timing_count % g_timing);
            if (depth > 1 && run >= depth && t->graph_n) {
                HIP_TRY(hipGraphLaunch(t->graph_n, stream));
                it += depth;
                g_timing_count += depth;
            } else {
                if (depth > 0) HIP_TRY(hipGraphLaunch(t->graph, stream));
                else HIP_TRY(launch_iteration(bt, prec, stream));
                ++it;
                ++g_timing_count;
            }
            continue;
        }
        ++it;
        ++g_timing_count;
        // a sampled iteration: direct launches bracketed by events
        TimedIter ti = {pooled_event(), pooled_event(), pooled_event(), pooled_event()};
        if (!ti.it0 || !ti.f0 || !ti.f1 || !ti.it1) return fail(KCM_E_DEVICE, "event creation failed");
        HIP_TRY(launch_iteration(bt, prec, stream, &ti));
        g_timed.push_back(ti);
    }
    if (n_iter > 0 && final) HIP_TRY(launch_final(bt, stream));
    return KCM_OK;
}

// kcm_step with g_mu held and the chains checked; st, if given, receives every
// chain's record after the call
kcm_status step_locked(kcm_chain *const *chains, int n_chains, int n_iter, int prec, hipStream_t stream,
                       std::vector<ChainStats> *st)
{
    kcm_status s;
    Table *t = nullptr;
    s = ensure_table(chains, n_chains, stream, &t);
    if (s != KCM_OK) return s;
    if ((s = iterate_locked(t, chains, n_chains, n_iter, prec, stream, false, true)) != KCM_OK) return s;
    if (st) return gather_stats(t, stream, *st);
    return KCM_OK;
}

}  // namespace

kcm_status kcm_step(kcm_chain *const *chains, int n_chains, int n_iter, void *hip_stream, kcm_step_report *reports)
{
    if (n_iter < 0) return fail(KCM_E_INVAL, "n_iter < 0");
    int prec = 0;
    kcm_status s = check_chains(chains, n_chains, &prec);
    if (s != KCM_OK) return s;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lock(g_mu);
    std::vector<ChainStats> st;
    s = step_locked(chains, n_chains, n_iter, prec, stream, reports ? &st : nullptr);
    if (s != KCM_OK || !reports) return s;
    kcm_status worst = KCM_OK;
    for (int i = 0; i < n_chains; ++i) {
        kcm_step_report &r = reports[i];
        r.e_elec = st[i].e_elec;
        r.e_vdw = st[i].e_vdw;
        r.e_cav = st[i].e_cav;
        r.max_tau = st[i].max_tau;
        r.max_dtheta = st[i].max_dtheta;
        r.iterations = st[i].iterations;
        r.status = st[i].status;
        r.converged = st[i].converged;
        if (st[i].status != 0 && worst == KCM_OK) worst = (kcm_status)st[i].status;
    }
    if (worst != KCM_OK) fail(worst, "a chain reported a failure status");
    return worst;
}

// ---------------------------------------------------------------------------
// kcm_step_noalloc: kcm_step with the batch table and the report records in a
// file-scope device array instead of memory the library allocates
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

constexpr size_t kNoallocAlign = 256;
constexpr size_t noalloc_round(size_t x) { return (x + kNoallocAlign - 1) & ~(kNoallocAlign - 1); }
constexpr int kNoallocChains = KCM_NOALLOC_MAX_CHAINS;
constexpr size_t kNaTab = noalloc_round(sizeof(ChainDev *) * kNoallocChains);  // chain descriptors
constexpr size_t kNaOff = noalloc_round(sizeof(int32_t) * (kNoallocChains + 1));  // one offset array
constexpr size_t kNaTable = kNaTab + 4 * kNaOff;  // descriptors, atom / block / joint-block / chunk offsets
constexpr size_t kNaStats = noalloc_round(sizeof(ChainStats) * kNoallocChains);
constexpr size_t kNoallocBytes = kNaTable + kNaStats;
static_assert(kNoallocBytes <= KCM_NOALLOC_SCRATCH_BYTES, "scratch size stated in kcm.h");
constexpr int kNoallocDevices = 64;

// The table and the gathered records of the last kcm_step_noalloc call on
// each device.  In host code `scratch` names a host-side stand-in: the
// device address of each device's copy comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

struct NoallocDevice {
    unsigned char *ptr = nullptr;        // this device's copy of scratch
    hipStream_t last = nullptr;          // stream of the last call that wrote the table
    bool used = false;
    int n_chains = 0;                    // the chain set the table holds
    const kcm_chain *chains[kNoallocChains];
    Batch batch{};
};
NoallocDevice g_noalloc[kNoallocDevices];
// host images, reused by every call (the calls are serialised by g_mu)
unsigned char g_noalloc_table[kNaTable];
ChainStats g_noalloc_stats[kNoallocChains];
const kcm_chain *g_noalloc_sorted[kNoallocChains];

// The device address of this device's scratch, looked up once per device.
kcm_status noalloc_device(int dev, NoallocDevice **out)
{
    if (dev < 0 || dev >= kNoallocDevices) return fail(KCM_E_INVAL, "kcm_step_noalloc: device index above 63");
    NoallocDevice &d = g_noalloc[dev];
    if (!d.ptr) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(KCM_E_DEVICE, "kcm_step_noalloc: hipGetSymbolAddress of the scratch array failed");
        d.ptr = static_cast<unsigned char *>(p);
    }
    *out = &d;
    return KCM_OK;
}

// The batch table of `chains` in the device's scratch (rewritten only when
// the chain set differs from the last call's).
kcm_status noalloc_table(NoallocDevice &d, kcm_chain *const *chains, int n_chains, hipStream_t stream)
{
    bool same = d.used && d.n_chains == n_chains;
    for (int i = 0; same && i < n_chains; ++i) same = d.chains[i] == chains[i];
    if (same) return KCM_OK;
    // the previous call's kernels, and its copy of the host image, are done
    // before either is overwritten
    if (d.used) {
        hipError_t e = hipStreamSynchronize(d.last);
        if (e != hipSuccess) return fail(KCM_E_DEVICE, "kcm_step_noalloc: synchronising the previous call failed");
    }
    ChainDev **tab = reinterpret_cast<ChainDev **>(g_noalloc_table);
    int32_t *off = reinterpret_cast<int32_t *>(g_noalloc_table + kNaTab);
    int32_t *blk = reinterpret_cast<int32_t *>(g_noalloc_table + kNaTab + kNaOff);
    int32_t *jblk = reinterpret_cast<int32_t *>(g_noalloc_table + kNaTab + 2 * kNaOff);
    int32_t *sblk = reinterpret_cast<int32_t *>(g_noalloc_table + kNaTab + 3 * kNaOff);
    long long total = 0, blocks = 0, jblocks = 0, sblocks = 0;
    int max_chunks = 1;
    for (int i = 0; i < n_chains; ++i) {
        tab[i] = chains[i]->d_desc;
        off[i] = (int32_t)total;
        blk[i] = (int32_t)blocks;
        jblk[i] = (int32_t)jblocks;
        sblk[i] = (int32_t)sblocks;
        total += chains[i]->n;
        blocks += (chains[i]->n + ATOM_BLOCK - 1) / ATOM_BLOCK;
        jblocks += chains[i]->njb;
        const int chunks = (chains[i]->h.cap_cells + SCAN_CHUNK - 1) / SCAN_CHUNK;
        sblocks += chunks;
        max_chunks = std::max(max_chunks, chunks);
    }
    if (total > std::numeric_limits<int32_t>::max() || sblocks > std::numeric_limits<int32_t>::max())
        return fail(KCM_E_INVAL, "too many atoms in one call");
    off[n_chains] = (int32_t)total;
    blk[n_chains] = (int32_t)blocks;
    jblk[n_chains] = (int32_t)jblocks;
    sblk[n_chains] = (int32_t)sblocks;
    d.used = false;  // until the copy below is queued
    hipError_t e = hipMemcpyAsync(d.ptr, g_noalloc_table, kNaTable, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return fail(KCM_E_DEVICE, "kcm_step_noalloc: copy of the batch table failed");
    Batch &b = d.batch;
    b.table = reinterpret_cast<ChainDev *const *>(d.ptr);
    b.atom_off = reinterpret_cast<const int32_t *>(d.ptr + kNaTab);
    b.blk_off = reinterpret_cast<const int32_t *>(d.ptr + kNaTab + kNaOff);
    b.jblk_off = reinterpret_cast<const int32_t *>(d.ptr + kNaTab + 2 * kNaOff);
    b.scan_off = reinterpret_cast<const int32_t *>(d.ptr + kNaTab + 3 * kNaOff);
    b.n_chains = n_chains;
    b.total_atoms = (int)total;
    b.total_blocks = (int)blocks;
    b.total_jblocks = (int)jblocks;
    b.total_scan_blocks = (int)sblocks;
    b.max_scan_chunks = max_chunks;
    for (int i = 0; i < n_chains; ++i) d.chains[i] = chains[i];
    d.n_chains = n_chains;
    d.used = true;
    d.last = stream;
    return KCM_OK;
}

}  // namespace

extern "C" {

kcm_status kcm_step_noalloc(kcm_chain *const *chains, int n_chains, int n_iter, void *hip_stream,
                            kcm_step_report *reports)
{
    if (n_iter < 0) return fail(KCM_E_INVAL, "n_iter < 0");
    if (!chains || n_chains < 1) return fail(KCM_E_INVAL, "no chains");
    if (n_chains > KCM_NOALLOC_MAX_CHAINS)
        return fail(KCM_E_INVAL, "kcm_step_noalloc takes at most KCM_NOALLOC_MAX_CHAINS (1024) chains");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(KCM_E_DEVICE, "hipGetDevice failed");
    for (int i = 0; i < n_chains; ++i) {
        if (!chains[i]) return fail(KCM_E_INVAL, "null chain handle");
        if (chains[i]->device != dev) return fail(KCM_E_INVAL, "chain lives on another device");
        if (chains[i]->h.precision != chains[0]->h.precision)
            return fail(KCM_E_INVAL, "chains of one call must share precision");
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lock(g_mu);
    std::copy(chains, chains + n_chains, g_noalloc_sorted);
    std::sort(g_noalloc_sorted, g_noalloc_sorted + n_chains);
    if (std::adjacent_find(g_noalloc_sorted, g_noalloc_sorted + n_chains) != g_noalloc_sorted + n_chains)
        return fail(KCM_E_INVAL, "a chain appears twice in one call");
    const int prec = chains[0]->h.precision;
    NoallocDevice *d = nullptr;
    kcm_status s = noalloc_device(dev, &d);
    if (s != KCM_OK) return s;
    if ((s = noalloc_table(*d, chains, n_chains, stream)) != KCM_OK) return s;
    if (d->last != stream) {
        // same chain set from another stream: the table stays, ordered after
        // the last writer's work
        hipError_t e = hipStreamSynchronize(d->last);
        if (e != hipSuccess) return fail(KCM_E_DEVICE, "kcm_step_noalloc: synchronising the previous call failed");
        d->last = stream;
    }
    const Batch &bt = d->batch;
    hipError_t e = hipSuccess;
    if (n_iter > 0) {
        bool boot = false;
        for (int i = 0; i < n_chains; ++i) boot = boot || chains[i]->boot;
        if (boot) {
            if ((e = launch_boot(bt, stream)) != hipSuccess) return fail(KCM_E_DEVICE, "kcm_step_noalloc: launch failed");
            for (int i = 0; i < n_chains; ++i) chains[i]->boot = false;
        }
        for (int it = 0; it < n_iter && e == hipSuccess; ++it) e = launch_iteration(bt, prec, stream);
        if (e == hipSuccess) e = launch_final(bt, stream);
        if (e != hipSuccess) return fail(KCM_E_DEVICE, "kcm_step_noalloc: launch failed");
    }
    if (!reports) return KCM_OK;
    ChainStats *dst = reinterpret_cast<ChainStats *>(d->ptr + kNaTable);
    if ((e = launch_stats_gather(bt, dst, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(g_noalloc_stats, dst, sizeof(ChainStats) * n_chains, hipMemcpyDeviceToHost, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess)
        return fail(KCM_E_DEVICE, "kcm_step_noalloc: reading the chains' records failed");
    kcm_status worst = KCM_OK;
    for (int i = 0; i < n_chains; ++i) {
        const ChainStats &c = g_noalloc_stats[i];
        kcm_step_report &r = reports[i];
        r.e_elec = c.e_elec;
        r.e_vdw = c.e_vdw;
        r.e_cav = c.e_cav;
        r.max_tau = c.max_tau;
        r.max_dtheta = c.max_dtheta;
        r.iterations = c.iterations;
        r.status = c.status;
        r.converged = c.converged;
        if (c.status != 0 && worst == KCM_OK) worst = (kcm_status)c.status;
    }
    if (worst != KCM_OK) fail(worst, "a chain reported a failure status");
    return worst;
}

kcm_status kcm_fold(kcm_chain *const *chains, int n_chains, double tol_dtheta, int max_iter, int check_every,
                    void *hip_stream, kcm_fold_result *results)
{
    int prec = 0;
    kcm_status s = check_chains(chains, n_chains, &prec);
    if (s != KCM_OK) return s;
    if (max_iter < 0 || check_every < 1) return fail(KCM_E_INVAL, "max_iter < 0 or check_every < 1");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lock(g_mu);
    const auto t0 = std::chrono::steady_clock::now();
    Table *t = nullptr;
    if ((s = ensure_table(chains, n_chains, stream, &t)) != KCM_OK) return s;
    std::vector<ChainStats> st;
    if ((s = gather_stats(t, stream, st)) != KCM_OK) return s;
    std::vector<int64_t> start(n_chains);
    for (int i = 0; i < n_chains; ++i) start[i] = st[i].iterations;
    HIP_TRY(launch_fold_control(t->batch, FOLD_BEGIN, tol_dtheta, (int64_t)max_iter, stream));
    int done = 0;
    while (done < max_iter) {
        const int k = std::min(check_every, max_iter - done);
        if ((s = step_locked(chains, n_chains, k, prec, stream, &st)) != KCM_OK) return s;
        done += k;
        bool any = false;
        for (int i = 0; i < n_chains; ++i) any = any || st[i].active;
        if (!any) break;
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (done == 0 && (s = gather_stats(t, stream, st)) != KCM_OK) return s;
    // leave the chains steppable again by kcm_step (ensure_table: the same
    // batch, so the table is still current)
    if ((s = ensure_table(chains, n_chains, stream, &t)) != KCM_OK) return s;
    HIP_TRY(launch_fold_control(t->batch, FOLD_END, 0.0, 0, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    kcm_status worst = KCM_OK;
    for (int i = 0; i < n_chains; ++i) {
        if (results) {
            results[i].iterations = st[i].iterations - start[i];
            results[i].converged = st[i].converged;
            results[i].status = st[i].status;
            results[i].seconds = secs;
        }
        if (st[i].status != 0 && worst == KCM_OK) worst = (kcm_status)st[i].status;
    }
    return worst;
}

kcm_status kcm_mc_minimize(kcm_chain *const *chains, int32_t n_chains, int32_t n_trials, int32_t n_descent, double kT,
                           const double *delta, const double *u, void *hip_stream, kcm_mc_result *results)
{
    int prec = 0;
    kcm_status s = check_chains(chains, n_chains, &prec);
    if (s != KCM_OK) return s;
    if (n_trials < 0 || n_descent < 0) return fail(KCM_E_INVAL, "n_trials < 0 or n_descent < 0");
    if (!(kT >= 0.0)) return fail(KCM_E_INVAL, "kT must be >= 0");
    if (n_trials > 0 && (!delta || !u)) return fail(KCM_E_INVAL, "null delta or u");
    if (n_trials > 0 && (!device_readable(delta) || !device_readable(u)))
        return fail(KCM_E_INVAL, "delta and u must be device memory");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lock(g_mu);
    Table *t = nullptr;
    if ((s = ensure_table(chains, n_chains, stream, &t)) != KCM_OK) return s;
    // per-chain offsets of the perturbations: chain c's [n_trials][J_c] block
    if ((s = upload_joint_offsets(t, chains, n_chains, n_trials, stream)) != KCM_OK) return s;
    const Batch &bt = t->batch;
    // the energy of the current angles: one evaluation, taken as the start
    HIP_TRY(launch_mc_propose(bt, MC_RESET, nullptr, nullptr, 0, stream));
    if ((s = iterate_locked(t, chains, n_chains, 1, prec, stream, true, false)) != KCM_OK) return s;
    HIP_TRY(launch_tau(bt, stream));
    HIP_TRY(launch_mc_decide(bt, MC_INIT, u, n_trials, 0, kT, stream));
    HIP_TRY(launch_mc_apply(bt, stream));
    for (int k = 0; k < n_trials; ++k) {
        // perturb, n_descent steps, and the evaluation of the reached angles
        HIP_TRY(launch_mc_propose(bt, MC_PROPOSE, delta, t->mc_off_dev, k, stream));
        if ((s = iterate_locked(t, chains, n_chains, n_descent + 1, prec, stream, true, false)) != KCM_OK) return s;
        HIP_TRY(launch_tau(bt, stream));
        HIP_TRY(launch_mc_decide(bt, MC_TRIAL, u, n_trials, k, kT, stream));
        HIP_TRY(launch_mc_apply(bt, stream));
    }
    std::vector<ChainStats> st;
    if ((s = gather_stats(t, stream, st)) != KCM_OK) return s;
    kcm_status worst = KCM_OK;
    for (int i = 0; i < n_chains; ++i) {
        // the angles are the accepted ones; positions and grid come anew
        chains[i]->boot = true;
        if (results) {
            kcm_mc_result &r = results[i];
            r.e_start = st[i].mc_e_start;
            r.e_accepted = st[i].mc_e_acc;
            r.e_best = st[i].mc_e_best;
            r.trials = st[i].mc_trials;
            r.accepted = st[i].mc_accepted;
            r.status = st[i].status;
            r.pad = 0;
        }
        if (st[i].status != 0 && worst == KCM_OK) worst = (kcm_status)st[i].status;
    }
    if (worst != KCM_OK) fail(worst, "a chain reported a failure status");
    return worst;
}

kcm_status kcm_mc_best_theta(const kcm_chain *c, void *hip_stream, double *theta)
{
    if (!c || !theta) return fail(KCM_E_INVAL, "null chain or theta");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(theta, c->h.mc_theta + c->J, 8 * (size_t)c->J, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return KCM_OK;
}

kcm_status kcm_get_state(const kcm_chain *c, void *hip_stream, double *theta, double *xyz, double *force, double *tau,
                         double *dtheta)
{
    if (!c) return fail(KCM_E_INVAL, "null chain");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipStreamSynchronize(s));
    if (theta) HIP_TRY(hipMemcpy(theta, c->h.theta, 8 * c->J, hipMemcpyDeviceToHost));
    if (tau) HIP_TRY(hipMemcpy(tau, c->h.tau, 8 * c->J, hipMemcpyDeviceToHost));
    if (dtheta) HIP_TRY(hipMemcpy(dtheta, c->h.dtheta, 8 * c->J, hipMemcpyDeviceToHost));
    if (xyz) {
        std::vector<double4> r(c->n);
        HIP_TRY(hipMemcpy(r.data(), c->h.r, 32 * (size_t)c->n, hipMemcpyDeviceToHost));
        for (int a = 0; a < c->n; ++a) {
            xyz[3 * a] = r[a].x;
            xyz[3 * a + 1] = r[a].y;
            xyz[3 * a + 2] = r[a].z;
        }
    }
    if (force) {
        std::vector<double4> fp(c->n);
        std::vector<long long> fc(3 * (size_t)c->n);
        HIP_TRY(hipMemcpy(fp.data(), c->h.f_pair, 32 * (size_t)c->n, hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(fc.data(), c->h.f_cav, 24 * (size_t)c->n, hipMemcpyDeviceToHost));
        for (int a = 0; a < c->n; ++a) {
            force[3 * a] = fp[a].x + (double)fc[3 * a] / FIX_SCALE;
            force[3 * a + 1] = fp[a].y + (double)fc[3 * a + 1] / FIX_SCALE;
            force[3 * a + 2] = fp[a].z + (double)fc[3 * a + 2] / FIX_SCALE;
        }
    }
    return KCM_OK;
}

kcm_status kcm_get_forces(const kcm_chain *c, void *hip_stream, double *f_pair, double *f_cav)
{
    if (!c) return fail(KCM_E_INVAL, "null chain");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
    if (f_pair) {
        std::vector<double4> fp(c->n);
        HIP_TRY(hipMemcpy(fp.data(), c->h.f_pair, 32 * (size_t)c->n, hipMemcpyDeviceToHost));
        for (int a = 0; a < c->n; ++a) {
            f_pair[3 * a] = fp[a].x;
            f_pair[3 * a + 1] = fp[a].y;
            f_pair[3 * a + 2] = fp[a].z;
        }
    }
    if (f_cav) {
        std::vector<long long> fc(3 * (size_t)c->n);
        HIP_TRY(hipMemcpy(fc.data(), c->h.f_cav, 24 * (size_t)c->n, hipMemcpyDeviceToHost));
        for (size_t k = 0; k < fc.size(); ++k) f_cav[k] = (double)fc[k] / FIX_SCALE;
    }
    return KCM_OK;
}

kcm_status kcm_get_atom_terms(const kcm_chain *c, void *hip_stream, double *e_elec, double *e_vdw, double *e_cav,
                              int32_t *n_exposed)
{
    if (!c) return fail(KCM_E_INVAL, "null chain");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
    std::vector<double4> e(c->n);
    HIP_TRY(hipMemcpy(e.data(), c->h.e_atom, 32 * (size_t)c->n, hipMemcpyDeviceToHost));
    for (int a = 0; a < c->n; ++a) {
        if (e_elec) e_elec[a] = e[a].x;
        if (e_vdw) e_vdw[a] = e[a].y;
        if (e_cav) e_cav[a] = e[a].z;
        if (n_exposed) n_exposed[a] = (int32_t)e[a].w;
    }
    return KCM_OK;
}

kcm_status kcm_set_theta(kcm_chain *c, const double *theta, void *hip_stream)
{
    if (!c || !theta) return fail(KCM_E_INVAL, "null chain or theta");
    std::vector<double> t(c->J);
    for (int j = 0; j < c->J; ++j) {
        if (!std::isfinite(theta[j])) return fail(KCM_E_INVAL, "theta not finite");
        double v = std::remainder(theta[j], 2.0 * kPi);
        if (v <= -kPi) v += 2.0 * kPi;
        t[j] = v;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(c->h.theta, t.data(), 8 * c->J, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    kcm_status st;
    if ((st = write_field(&c->h.stats->converged, 0, s)) != KCM_OK) return st;
    if ((st = write_field(&c->h.stats->status, 0, s)) != KCM_OK) return st;
    if ((st = write_field(&c->h.stats->nbr_overflow, 0, s)) != KCM_OK) return st;
    if ((st = write_field(&c->h.stats->need_grid, 1, s)) != KCM_OK) return st;
    if ((st = write_field(&c->h.stats->pending_post, 0, s)) != KCM_OK) return st;
    if ((st = write_field(&c->h.stats->run, 1, s)) != KCM_OK) return st;
    if ((st = write_field(&c->h.stats->grid_bad, 0, s)) != KCM_OK) return st;
    c->boot = true;
    return write_field(&c->h.stats->active, 1, s);
}

kcm_status kcm_set_theta_batch(kcm_chain *const *chains, int32_t n_chains, const double *theta, void *hip_stream)
{
    int prec = 0;
    kcm_status s = check_chains(chains, n_chains, &prec);
    if (s != KCM_OK) return s;
    if (!theta) return fail(KCM_E_INVAL, "null theta");
    if (!device_readable(theta)) return fail(KCM_E_INVAL, "theta must be device memory");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    std::lock_guard<std::mutex> lock(g_mu);
    Table *t = nullptr;
    if ((s = ensure_table(chains, n_chains, stream, &t)) != KCM_OK) return s;
    if ((s = upload_joint_offsets(t, chains, n_chains, 1, stream)) != KCM_OK) return s;
    HIP_TRY(launch_set_theta(t->batch, theta, t->mc_off_dev, stream));
    for (int i = 0; i < n_chains; ++i) chains[i]->boot = true;
    return KCM_OK;
}

kcm_status kcm_set_limits(kcm_chain *c, double tol_dtheta, int64_t max_iterations, void *hip_stream)
{
    if (!c || !std::isfinite(tol_dtheta)) return fail(KCM_E_INVAL, "null chain or tol not finite");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    kcm_status st;
    if ((st = write_field(&c->h.stats->tol, tol_dtheta, s)) != KCM_OK) return st;
    return write_field(&c->h.stats->iter_limit,
                       max_iterations > 0 ? max_iterations : std::numeric_limits<int64_t>::max(), s);
}

kcm_status kcm_get_cells(const kcm_chain *c, void *hip_stream, int32_t *dims, double *cell_size, double *origin,
                         int32_t *n_cells, int32_t *order, int32_t *cell_start, int32_t cell_start_capacity)
{
    if (!c) return fail(KCM_E_INVAL, "null chain");
    HIP_TRY(hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
    Grid g;
    HIP_TRY(hipMemcpy(&g, c->h.grid, sizeof g, hipMemcpyDeviceToHost));
    if (dims) for (int k = 0; k < 3; ++k) dims[k] = g.dims[k];
    if (cell_size) *cell_size = g.cell;
    if (origin) for (int k = 0; k < 3; ++k) origin[k] = g.origin[k];
    if (n_cells) *n_cells = g.n_cells;
    if (order) HIP_TRY(hipMemcpy(order, c->h.s_idx, 4 * (size_t)c->n, hipMemcpyDeviceToHost));
    if (cell_start) {
        if (cell_start_capacity < g.n_cells + 1) return fail(KCM_E_INVAL, "cell_start_capacity too small");
        HIP_TRY(hipMemcpy(cell_start, c->h.cell_start, 4 * ((size_t)g.n_cells + 1), hipMemcpyDeviceToHost));
    }
    return KCM_OK;
}

kcm_status kcm_set_graphs(int iterations)
{
    if (iterations < 0 || iterations > kMaxGraphDepth) return fail(KCM_E_INVAL, "iterations per graph must be in 0..64");
    std::lock_guard<std::mutex> lock(g_mu);
    g_graphs = iterations;
    return KCM_OK;
}

kcm_status kcm_set_force_variant(int variant)
{
    if (variant < 0 || variant >= FORCE_SHAPE_COUNT) return fail(KCM_E_INVAL, "force variant out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    g_force_shape = variant;
    return KCM_OK;
}

kcm_status kcm_set_timing(int every)
{
    if (every < 0) return fail(KCM_E_INVAL, "every < 0");
    std::lock_guard<std::mutex> lock(g_mu);
    g_timing = every;
    g_timing_count = 0;
    return KCM_OK;
}

kcm_status kcm_get_timing(double *force_ms, int64_t *force_launches, double *iter_ms, int64_t *iterations, int reset)
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &t : g_timed) {
        HIP_TRY(hipEventSynchronize(t.it1));
        float a = 0.f, b = 0.f;
        HIP_TRY(hipEventElapsedTime(&a, t.f0, t.f1));
        HIP_TRY(hipEventElapsedTime(&b, t.it0, t.it1));
        g_force_ms += a;
        g_iter_ms += b;
        g_force_n += 1;
        g_iter_n += 1;
        g_event_pool.push_back(t.it0);
        g_event_pool.push_back(t.f0);
        g_event_pool.push_back(t.f1);
        g_event_pool.push_back(t.it1);
    }
    g_timed.clear();
    if (force_ms) *force_ms = g_force_ms;
    if (force_launches) *force_launches = g_force_n;
    if (iter_ms) *iter_ms = g_iter_ms;
    if (iterations) *iterations = g_iter_n;
    if (reset) {
        g_force_ms = g_iter_ms = 0.0;
        g_force_n = g_iter_n = 0;
    }
    return KCM_OK;
}

kcm_status kcm_chain_free(kcm_chain *c)
{
    if (!c) return fail(KCM_E_INVAL, "null chain");
    std::lock_guard<std::mutex> lock(g_mu);
    for (auto &t : g_tables) {
        for (auto *x : t.chains)
            if (x == c) {
                t.chains.clear();  // forces a rebuild of this table on next use
                if (t.graph) {
                    (void)hipGraphExecDestroy(t.graph);
                    t.graph = nullptr;
                }
                if (t.graph_n) {
                    (void)hipGraphExecDestroy(t.graph_n);
                    t.graph_n = nullptr;
                }
                break;
            }
    }
    delete c;
    return KCM_OK;
}

}  // extern "C"
