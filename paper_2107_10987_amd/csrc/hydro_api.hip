// Host side of the C ABI declared in include/hydro.h: handle and workspace
// management, argument validation, stage sequencing and the octree ghost map.

#include "hydro_common.h"
#include "mlp_common.h"
#include "../../include/hydro.h"

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

using namespace hydro;

constexpr int NSIDE = 3;   // side streams for the launches of a stage

struct hydro_t {
    hydro_params p;
    int device;
    double *U1 = nullptr;      // first-stage state [max_leaves][7][512]
    double *U2 = nullptr;      // second-stage state of three-stage steps
    int rk = 2;
    int ts = 0, lg = 3;        // 8^3 blocks per leaf (log2), leaf edge (log2)
    double *dscr = nullptr;    // column walk: [max_leaves][3][7][512]
    int *queue = nullptr;      // persistent launches: [1 + NSIDE][QUEUE_INTS], one per stream
    // the launches of one stage run on the caller's stream and NSIDE side
    // streams (default priority), forked from and joined back to it by events
    hipStream_t side[NSIDE] = {};
    hipEvent_t fork_ev = nullptr;
    hipEvent_t join_ev[NSIDE] = {};
    int *leaf_done = nullptr;  // [max_leaves]
    double *tile_amax = nullptr;  // [max_leaves][3]
    double *bflux = nullptr;   // flux correction: [max_leaves][6][7][64]
    int num_cu = 0;
    int32_t table[HYDRO_NBUCKET];  // schedule per launch-size bucket (HYDRO_SCHED_AUTO)
    int32_t multi_sched = -1;      // stages of several concurrent launches: one schedule for all (-1:
                                   // table; MULTI_MERGE: one launch over the whole partition)
    bool table_loaded = false;
    std::string arch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    // learned reconstruction
    mlp::MlpTrain mt{};
    int mlp_batch = 0;
    int adam_t = 0;
    bool mlp_loaded = false;
    float *mlp_off = nullptr;      // [max_leaves][7][26][896] point values as offsets
    uint8_t *mlp_ok = nullptr;     // [max_leaves][896]
    unsigned long long *fb_count = nullptr;
    int64_t mlp_cells = 0;
    int64_t graph_mlp_cells = 0;   // cells the captured graph reconstructs per replay
    std::vector<void *> mlp_bufs;  // everything allocated for the network
    double *amax = nullptr;    // per-block signal speeds [max_leaves << ts]
    Status *status = nullptr;  // device status word
    hipStream_t last_stream = nullptr;
    std::string err;
    // stage-kernel timing
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pairs (start, stop)
    size_t ev_used = 0;          // pairs recorded since the last report
};

namespace {

thread_local std::string g_create_err;

int fail(hydro_t *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    else g_create_err = msg;
    return code;
}

int hip_fail(hydro_t *h, hipError_t e, const char *what) {
    return fail(h, HYDRO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Padded index of each ghost slot in raster order (k, j, i over -3..10,
// interior skipped); the same order as the ghost map.
std::vector<uint16_t> ghost_table() {
    std::vector<uint16_t> t;
    t.reserve(NG);
    for (int k = -GW; k < NX + GW; ++k)
        for (int j = -GW; j < NX + GW; ++j)
            for (int i = -GW; i < NX + GW; ++i) {
                const bool in = i >= 0 && i < NX && j >= 0 && j < NX && k >= 0 && k < NX;
                if (!in) t.push_back((uint16_t)(((k + GW) * PB + (j + GW)) * PB + (i + GW)));
            }
    return t;
}

// Ghost slot of each padded cell (-1 for interior cells), the inverse of
// ghost_table().
std::vector<int16_t> pad_ghost_table() {
    std::vector<int16_t> t(NP, -1);
    const std::vector<uint16_t> g = ghost_table();
    for (int s = 0; s < NG; ++s) t[g[s]] = (int16_t)s;
    return t;
}

std::once_flag g_table_once[64];
hipError_t g_table_err[64];

hipError_t ensure_ghost_table(int dev) {
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::call_once(g_table_once[dev], [dev] {
        std::vector<uint16_t> t = ghost_table();
        g_table_err[dev] = hydro_upload_ghost_table(t.data());
        if (g_table_err[dev] == hipSuccess) {
            std::vector<int16_t> pg = pad_ghost_table();
            g_table_err[dev] = hydro_mlp_upload_pad_ghost(pg.data());
        }
    });
    return g_table_err[dev];
}

int check_grid(hydro_t *h, const hydro_grid *g) {
    if (!h) return HYDRO_EINVAL;
    if (!g) return fail(h, HYDRO_EINVAL, "grid is NULL");
    if (g->n <= 0) return fail(h, HYDRO_EINVAL, "grid has no leaves");
    if (g->n > h->p.max_leaves)
        return fail(h, HYDRO_ENOMEM, "grid has " + std::to_string(g->n) + " leaves, workspace holds " +
                                         std::to_string(h->p.max_leaves));
    if (!g->dx || !g->origin || !g->ghost_map) return fail(h, HYDRO_EINVAL, "null dx/origin/ghost_map");
    if (!(g->gamma > 1.0) || !isfinite(g->gamma)) return fail(h, HYDRO_EINVAL, "gamma must be > 1");
    if (!isfinite(g->omega)) return fail(h, HYDRO_EINVAL, "omega must be finite");
    if (h->p.reflux) {
        if (!g->face_flags) return fail(h, HYDRO_EINVAL, "reflux needs g->face_flags (hydro_reflux_map)");
        if (g->n_reflux < 0 || g->n_reflux > (g->n << h->ts)) return fail(h, HYDRO_EINVAL, "n_reflux out of range");
        if (g->n_reflux > 0 && !g->reflux) return fail(h, HYDRO_EINVAL, "reflux list is NULL");
    } else if (g->face_flags || g->n_reflux) {
        return fail(h, HYDRO_EINVAL, "grid carries reflux lists but the handle was created without reflux");
    }
    if (g->n_prolong < 0 || (g->n_prolong > 0 && !g->prolong))
        return fail(h, HYDRO_EINVAL, "bad prolongation table");
    if (g->n_launch < 0) return fail(h, HYDRO_EINVAL, "n_launch < 0");
    if (g->n_launch > 0) {
        if (!g->launch_off) return fail(h, HYDRO_EINVAL, "launch_off is NULL");
        if (g->launch_off[0] != 0 || g->launch_off[g->n_launch] != g->n)
            return fail(h, HYDRO_EINVAL, "launch_off must run from 0 to n");
        for (int b = 0; b < g->n_launch; ++b)
            if (g->launch_off[b + 1] < g->launch_off[b])
                return fail(h, HYDRO_EINVAL, "launch_off must be non-decreasing");
    }
    return HYDRO_OK;
}

bool aligned8(const void *p) { return ((uintptr_t)p & 7u) == 0; }

// Leaf lookup by (level, leaf coordinates) of a validated tree.
struct TreeIndex {
    const hydro_tree *t = nullptr;
    int lmax = 0;
    std::unordered_map<uint64_t, int32_t> owner;
    static uint64_t key(int l, int64_t x, int64_t y, int64_t z) {
        return ((uint64_t)l << 60) | ((uint64_t)z << 40) | ((uint64_t)y << 20) | (uint64_t)x;
    }
    int build(const hydro_tree *tree) {
        t = tree;
        if (!t || !t->level || !t->coord || t->n <= 0) return fail(nullptr, HYDRO_EINVAL, "null or empty tree");
        if (t->leaf_edge != 0 && t->leaf_edge != 8 && t->leaf_edge != 16)
            return fail(nullptr, HYDRO_EINVAL, "leaf_edge must be 8 or 16");
        if ((int64_t)t->n * (t->leaf_edge == 16 ? 4096 : NC) > INT32_MAX)
            return fail(nullptr, HYDRO_EINVAL, "too many leaves for int32 cell ids");
        for (int a = 0; a < 3; ++a)
            if (t->nb[a] <= 0 || (t->bc[a] != 0 && t->bc[a] != 1))
                return fail(nullptr, HYDRO_EINVAL, "bad nb/bc");
        for (int i = 0; i < t->n; ++i) {
            if (t->level[i] < 0 || t->level[i] > 20) return fail(nullptr, HYDRO_EINVAL, "level out of range");
            lmax = t->level[i] > lmax ? t->level[i] : lmax;
        }
        owner.reserve((size_t)t->n * 2);
        for (int i = 0; i < t->n; ++i) {
            const int32_t *c = t->coord + 3 * (size_t)i;
            const int l = t->level[i];
            for (int a = 0; a < 3; ++a)
                if (c[a] < 0 || (int64_t)c[a] >= ((int64_t)t->nb[a] << l))
                    return fail(nullptr, HYDRO_EINVAL, "leaf outside the box");
            if (!owner.emplace(key(l, c[0], c[1], c[2]), i).second)
                return fail(nullptr, HYDRO_EINVAL, "duplicate leaf");
        }
        return HYDRO_OK;
    }
    // the leaf at level l with leaf coordinates (x, y, z), or -1
    int32_t leaf(int l, int64_t x, int64_t y, int64_t z) const {
        auto it = owner.find(key(l, x, y, z));
        return it == owner.end() ? -1 : it->second;
    }
};

int set_device(hydro_t *h) {
    hipError_t e = hipSetDevice(h->device);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "hipSetDevice");
}

// Launch one stage over all leaves, split as the grid asks.
int bucket_of(int nleaf) {
    int b = 0;
    while ((2 << b) <= nleaf && b < HYDRO_NBUCKET - 1) ++b;
    return b;
}

// The autotuner's choice for a grid's launch partition that replaces it by
// one launch over all its leaves (the ranges are consecutive, from 0 to n),
// with the per-size table's schedule.
constexpr int MULTI_MERGE = 5;

// Schedule of a launch of nleaf leaves.
int resolve_schedule(const hydro_t *h, int nleaf, bool concurrent) {
    if (h->p.schedule != HYDRO_SCHED_AUTO) return h->p.schedule;
    if (concurrent && h->multi_sched >= 0 && h->multi_sched != MULTI_MERGE) return h->multi_sched;
    if (h->table_loaded) return h->table[bucket_of(nleaf)];
    // built-in rule: spread small launches over (leaf, axis) tiles so they
    // still occupy most compute units; otherwise a workgroup per leaf
    return (3 * nleaf <= h->num_cu) ? HYDRO_SCHED_TILED : HYDRO_SCHED_COLUMN;
}

void set_schedule(StageArgs &a, int sched) {
    switch (sched) {
    case HYDRO_SCHED_FACE: a.kernel = KERNEL_FACE; a.tiles = 1; break;
    case HYDRO_SCHED_PERSISTENT: a.kernel = KERNEL_PERSISTENT; a.tiles = 1; break;
    case HYDRO_SCHED_TILED: a.kernel = KERNEL_PERSISTENT; a.tiles = 3; break;
    default: a.kernel = KERNEL_COLUMN; a.tiles = 1; break;
    }
}

int run_stage(hydro_t *h, const hydro_grid *g, int stage, double dt, const double *Uin,
              const double *Un, double *Uout, double *amax, int accumulate,
              const double *dt_dev = nullptr, bool allow_timing = true) {
    if (h->p.recon == 1 && !h->mlp_loaded)
        return fail(h, HYDRO_EINVAL, "learned reconstruction needs hydro_mlp_load first");
    StageArgs a;
    a.Uin = Uin;
    a.Un = Un;
    a.Uout = Uout;
    a.dx = g->dx;
    a.origin = g->origin;
    a.gmap = g->ghost_map;
    a.amax = amax;
    a.status = h->status;
    a.ph = Phys{g->gamma, g->omega, h->p.eta1, h->p.eta2};
    a.dt = dt;
    a.stage = stage;
    a.amax_accumulate = accumulate;
    a.last = stage == h->rk;
    a.ca = 0.0;
    a.cb = 1.0;
    if (stage >= 2) {
        a.ca = h->rk == 2 ? 0.5 : (stage == 2 ? 0.75 : 1.0 / 3.0);
        a.cb = h->rk == 2 ? 0.5 : (stage == 2 ? 0.25 : 2.0 / 3.0);
    }
    a.dscr = h->dscr;
    a.dt_dev = dt_dev;
    a.queue = h->queue;
    a.leaf_done = h->leaf_done;
    a.tile_amax = h->tile_amax;
    a.grid_limit = h->num_cu;
    a.mlp_off = nullptr;
    a.mlp_ok = nullptr;
    a.mlp_alias = nullptr;
    a.centre_only = h->p.scheme == 1;
    a.ts = h->ts;
    a.lg = h->lg;
    a.prolong = g->prolong;
    a.n_prolong = g->n_prolong;
    const bool reflux = h->p.reflux && stage != 0;
    a.face_flags = reflux ? g->face_flags : nullptr;
    a.bflux = reflux ? h->bflux : nullptr;
    hipStream_t s = (hipStream_t)g->stream;
    h->last_stream = s;
    // the tuned merge of the partition: one launch over leaves 0..n
    const bool merge = g->n_launch > 1 && h->p.schedule == HYDRO_SCHED_AUTO && h->multi_sched == MULTI_MERGE;
    const int nlaunch = merge ? 0 : g->n_launch;
    const int nb = nlaunch > 0 ? nlaunch : 1;
    // the launches of a stage read the same input and write disjoint blocks:
    // they run concurrently on up to 1 + NSIDE streams (the caller's first),
    // each with its own persistent-queue counters, and the caller's stream
    // waits for all of them before anything that follows
    int nonempty = 0;
    for (int b = 0; b < nb; ++b)
        nonempty += (nlaunch > 0 ? g->launch_off[b + 1] - g->launch_off[b] : g->n) > 0;
    const int nst = nonempty < 1 + NSIDE ? (nonempty > 0 ? nonempty : 1) : 1 + NSIDE;
    if (nst > 1) {
        hipError_t e = hipEventRecord(h->fork_ev, s);
        for (int i = 0; i < nst - 1 && e == hipSuccess; ++i) e = hipStreamWaitEvent(h->side[i], h->fork_ev, 0);
        if (e != hipSuccess) return hip_fail(h, e, "stream fork");
    }
    int k = 0;   // non-empty launches so far
    for (int b = 0; b < nb; ++b) {
        // launches count 8^3 blocks: 2^ts per leaf
        const int l0 = nlaunch > 0 ? g->launch_off[b] : 0;
        const int nl = nlaunch > 0 ? g->launch_off[b + 1] - l0 : g->n;
        a.leaf0 = l0 << h->ts;
        a.nleaf = nl << h->ts;
        if (a.nleaf == 0) continue;
        const int j = k++ % nst;
        const hipStream_t st = j == 0 ? s : h->side[j - 1];
        a.queue = h->queue + QUEUE_INTS * j;
        set_schedule(a, resolve_schedule(h, a.nleaf, nst > 1));
        if (h->p.recon == 1) {
            // the network's point values and per-cell verdicts for this launch
            mlp::MlpInfer m{};
            m.U = Uin;
            m.gmap = g->ghost_map;
            m.wbi = h->mt.wbi;
            m.bi = h->mt.bi;
            m.off = h->mlp_off;
            m.cell_ok = h->mlp_ok;
            m.fb_count = h->fb_count;
            m.leaf0 = a.leaf0;
            m.ts = h->ts;
            m.lg = h->lg;
            m.prolong = g->prolong;
            m.n_prolong = g->n_prolong;
            m.alias = g->mlp_alias;
            hipError_t e = hydro_mlp_launch_infer(m, a.nleaf, st);
            if (e != hipSuccess) return hip_fail(h, e, "inference launch");
            h->mlp_cells += (int64_t)a.nleaf * NC;
            a.mlp_off = h->mlp_off;
            a.mlp_ok = h->mlp_ok;
            a.mlp_alias = g->mlp_alias;
            if (a.kernel == KERNEL_FACE) a.kernel = KERNEL_COLUMN;   // the face walk has no learned variant
        }
        const bool rec = allow_timing && h->timing && 2 * (h->ev_used + 1) <= h->ev.size();
        if (rec) (void)hipEventRecord(h->ev[2 * h->ev_used], st);
        hipError_t e = hydro_launch_stage(a, st);
        if (e != hipSuccess) return hip_fail(h, e, "stage launch");
        if (rec) (void)hipEventRecord(h->ev[2 * h->ev_used++ + 1], st);
    }
    for (int i = 0; i < nst - 1; ++i) {
        hipError_t e = hipEventRecord(h->join_ev[i], h->side[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, h->join_ev[i], 0);
        if (e != hipSuccess) return hip_fail(h, e, "stream join");
    }
    if (reflux && g->n_reflux > 0) {
        // after every launch of the stage: the finer leaves' fluxes are all kept
        RefluxArgs r;
        r.U = Uout;
        r.bflux = h->bflux;
        r.entries = g->reflux;
        r.dx = g->dx;
        r.dt = dt;
        r.dt_dev = dt_dev;
        r.cb = a.cb;
        r.last = a.last;
        r.ph = a.ph;
        r.status = h->status;
        r.ts = h->ts;
        r.lg = h->lg;
        hipError_t e = hydro_launch_reflux(r, g->n_reflux, s);
        if (e != hipSuccess) return hip_fail(h, e, "reflux launch");
    }
    return HYDRO_OK;
}

int read_status(hydro_t *h, hipStream_t s) {
    Status st;
    hipError_t e = hipMemcpyAsync(&st, h->status, sizeof(Status), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(h, e, "status read");
    if (st.flag) {
        e = hipMemsetAsync(h->status, 0, sizeof(Status), s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "status reset");
        static const char *names[NF] = {"rho", "sx", "sy", "sz", "egas", "tau", "spc"};
        char buf[160];
        snprintf(buf, sizeof buf, "non-physical %s at leaf %d cell %d",
                 (st.field >= 0 && st.field < NF) ? names[st.field] : "value", st.leaf, st.cell);
        return fail(h, HYDRO_ENONPHYS, buf);
    }
    return HYDRO_OK;
}

// Autotune table as JSON: {"arch": "...", "schedule": [b0, ..., b15]}.
int load_table(hydro_t *h, const char *path) {
    std::ifstream f(path);
    if (!f) return fail(h, HYDRO_EINVAL, std::string("cannot read tune cache ") + path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string t = ss.str();
    const size_t k = t.find("\"schedule\"");
    const size_t o = k == std::string::npos ? k : t.find('[', k);
    if (o == std::string::npos) return fail(h, HYDRO_EINVAL, "tune cache has no schedule list");
    const size_t a = t.find("\"arch\"");
    if (a != std::string::npos) {
        const size_t q0 = t.find('"', t.find(':', a) + 1), q1 = t.find('"', q0 + 1);
        if (q0 != std::string::npos && q1 != std::string::npos && t.substr(q0 + 1, q1 - q0 - 1) != h->arch)
            return fail(h, HYDRO_EINVAL, "tune cache was made for another GPU");
    }
    size_t pos = o + 1;
    for (int b = 0; b < HYDRO_NBUCKET; ++b) {
        char *end = nullptr;
        const long v = strtol(t.c_str() + pos, &end, 10);
        if (end == t.c_str() + pos || v < HYDRO_SCHED_FACE || v > HYDRO_SCHED_TILED)
            return fail(h, HYDRO_EINVAL, "bad schedule list in tune cache");
        h->table[b] = (int32_t)v;
        pos = (size_t)(end - t.c_str());
        while (pos < t.size() && (t[pos] == ',' || t[pos] == ' ' || t[pos] == '\n')) ++pos;
    }
    h->table_loaded = true;
    h->multi_sched = -1;
    const size_t c = t.find("\"concurrent\"");
    if (c != std::string::npos) {
        const size_t colon = t.find(':', c);
        char *end = nullptr;
        const long v = colon == std::string::npos ? -2 : strtol(t.c_str() + colon + 1, &end, 10);
        if (v < -1 || v == HYDRO_SCHED_AUTO || (v > HYDRO_SCHED_TILED && v != MULTI_MERGE))
            return fail(h, HYDRO_EINVAL, "bad concurrent schedule in tune cache");
        h->multi_sched = (int32_t)v;
    }
    return HYDRO_OK;
}

int save_table(hydro_t *h, const char *path) {
    std::ofstream f(path);
    if (!f) return fail(h, HYDRO_EINVAL, std::string("cannot write tune cache ") + path);
    f << "{\"arch\": \"" << h->arch << "\", \"schedule\": [";
    for (int b = 0; b < HYDRO_NBUCKET; ++b) f << (b ? ", " : "") << h->table[b];
    f << "], \"concurrent\": " << h->multi_sched << "}\n";
    return f.good() ? HYDRO_OK : fail(h, HYDRO_EINVAL, "tune cache write failed");
}

// All stages of one step, in place on g->U; per-leaf speeds accumulate in h->amax.
int run_stages(hydro_t *h, const hydro_grid *g, double dt, const double *dt_dev, bool allow_timing) {
    int rc;
    if ((rc = run_stage(h, g, 1, dt, g->U, g->U, h->U1, h->amax, 0, dt_dev, allow_timing))) return rc;
    if (h->rk == 2) return run_stage(h, g, 2, dt, h->U1, g->U, g->U, h->amax, 1, dt_dev, allow_timing);
    if ((rc = run_stage(h, g, 2, dt, h->U1, g->U, h->U2, h->amax, 1, dt_dev, allow_timing))) return rc;
    return run_stage(h, g, 3, dt, h->U2, g->U, g->U, h->amax, 1, dt_dev, allow_timing);
}

// All stages and the next dt, on the device.
int run_step_dev(hydro_t *h, const hydro_grid *g, double cfl, double *dt_dev, bool allow_timing) {
    int rc;
    if ((rc = run_stages(h, g, 0.0, dt_dev, allow_timing))) return rc;
    hipError_t e = hydro_launch_dt(g->dx, h->amax, g->n, h->ts, cfl, dt_dev, (hipStream_t)g->stream);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "dt launch");
}

// Per-block signal speeds of the handle -> per-leaf values in out (device).
int leaf_amax(hydro_t *h, const hydro_grid *g, double *out) {
    hipError_t e = hydro_launch_amax_leaves(h->amax, h->ts, g->n, out, (hipStream_t)g->stream);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "amax reduction");
}

template <class T>
hipError_t mlp_alloc(hydro_t *h, T **p, size_t count) {
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e == hipSuccess) {
        h->mlp_bufs.push_back((void *)*p);
        e = hipMemset((void *)*p, 0, count * sizeof(T));
    }
    return e;
}

// Network parameters, Adam state and training workspace (always: a few MB),
// plus the per-leaf inference outputs when the learned path is on.
hipError_t alloc_mlp(hydro_t *h, size_t nleaves) {
    const size_t B = h->p.mlp_batch > 0 ? (size_t)h->p.mlp_batch : 4096;
    h->mlp_batch = (int)B;
    mlp::MlpTrain &t = h->mt;
    hipError_t e = mlp_alloc(h, &t.par, mlp::NPAR);
    if (e == hipSuccess) e = mlp_alloc(h, &t.m, mlp::NPAR);
    if (e == hipSuccess) e = mlp_alloc(h, &t.v, mlp::NPAR);
    if (e == hipSuccess) e = mlp_alloc(h, &t.grad, mlp::NPAR);
    if (e == hipSuccess) e = mlp_alloc(h, &t.wb, mlp::WB_SIZE);
    if (e == hipSuccess) e = mlp_alloc(h, &t.wbT, mlp::WBT_SIZE);
    if (e == hipSuccess) e = mlp_alloc(h, &t.wbi, mlp::WBI_SIZE);
    if (e == hipSuccess) e = mlp_alloc(h, &t.bi, mlp::BI_SIZE);
    if (e == hipSuccess) e = mlp_alloc(h, &t.xb, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.a1, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.a2, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.dz1, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.dz2, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.z1, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.z2, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.dz1f, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.dz2f, B * 64);
    if (e == hipSuccess) e = mlp_alloc(h, &t.y, B * 32);
    if (e == hipSuccess) e = mlp_alloc(h, &t.dy, B * 32);
    if (e == hipSuccess) e = mlp_alloc(h, &t.loss_rows, B);
    if (e == hipSuccess) e = mlp_alloc(h, &t.gpart, (size_t)mlp::WG_SLICES * mlp::NPAR);
    if (e == hipSuccess) e = mlp_alloc(h, &h->fb_count, 1);
    if (e == hipSuccess && h->p.recon == 1) {
        e = mlp_alloc(h, &h->mlp_off, nleaves * mlp::NSLOT * NF * 26);
        if (e == hipSuccess) e = mlp_alloc(h, &h->mlp_ok, nleaves * mlp::NSLOT);
    }
    return e;
}

int check_batch(hydro_t *h, const void *X, int B) {
    if (!X) return fail(h, HYDRO_EINVAL, "null network input");
    if (B <= 0 || B > h->mlp_batch)
        return fail(h, HYDRO_EINVAL, "batch must be in 1.." + std::to_string(h->mlp_batch));
    return HYDRO_OK;
}


// Ghost maps of every tile of every leaf; with `table` non-NULL, ghost cells
// inside a coarser leaf get a linear-prolongation row instead of a copy.
int build_ghost_map(const hydro_tree *t, int32_t *map, int32_t *table, int32_t capacity,
                    int32_t *n_table) {
    if (!map) return fail(nullptr, HYDRO_EINVAL, "null map");
    TreeIndex ti;
    int rc = ti.build(t);
    if (rc) return rc;
    const int lmax = ti.lmax;
    const int lg = t->leaf_edge == 16 ? 4 : 3;   // build() accepted 0, 8 or 16
    const int64_t E = (int64_t)1 << lg;
    const int tiles = t->leaf_edge == 16 ? 8 : 1;
    const bool linear = n_table != nullptr;
    if (linear && (int64_t)t->n * E * E * E >= PROLONG_BASE)
        return fail(nullptr, HYDRO_EINVAL, "too many leaves for a prolongation map");
    // the leaf at level l holding global cell g (cells of that level), and
    // the cell's index inside that leaf
    auto find = [&](int l, const int64_t g[3]) -> int32_t { return ti.leaf(l, g[0] >> lg, g[1] >> lg, g[2] >> lg); };
    auto local = [&](const int64_t g[3]) -> int32_t {
        return (int32_t)((((g[2] & (E - 1)) * E + (g[1] & (E - 1))) * E) + (g[0] & (E - 1)));
    };
    const int32_t cells = (int32_t)(E * E * E);
    // wrap or clamp global cell g of level l into the box, in place
    auto fold = [&](int l, int64_t g[3]) {
        for (int a = 0; a < 3; ++a) {
            const int64_t nc = E * t->nb[a] << l;
            if (g[a] < 0 || g[a] >= nc) {
                if (t->bc[a] == 0) g[a] = ((g[a] % nc) + nc) % nc;
                else g[a] = g[a] < 0 ? 0 : nc - 1;
            }
        }
    };
    // map entry of level-l cell g: a copy from the leaf covering it at level
    // <= l (injection), else the mean of its 2x2x2 cells one level finer;
    // *covering = level of the covering leaf, or l + 1
    std::string err;
    auto entry = [&](int l, const int64_t g[3], int *covering) -> int64_t {
        for (int lc = l; lc >= 0; --lc) {
            const int64_t gc[3] = {g[0] >> (l - lc), g[1] >> (l - lc), g[2] >> (l - lc)};
            const int32_t o = find(lc, gc);
            if (o >= 0) {
                *covering = lc;
                return (int64_t)o * cells + local(gc);
            }
        }
        const int64_t gf[3] = {2 * g[0], 2 * g[1], 2 * g[2]};
        const int32_t o = (l < lmax) ? find(l + 1, gf) : -1;
        if (o < 0) return INT64_MIN;
        *covering = l + 1;
        return -((int64_t)o * cells + local(gf)) - 1;
    };
    int32_t rows = 0;
    for (int i = 0; i < t->n; ++i) {
        const int l = t->level[i];
        const int32_t *c = t->coord + 3 * (size_t)i;
        for (int tile = 0; tile < tiles; ++tile) {
            const int to[3] = {8 * (tile & 1), 8 * ((tile >> 1) & 1), 8 * (tile >> 2)};
            int32_t *m = map + ((size_t)i * tiles + tile) * NG;
            int s = 0;
            for (int k = -GW; k < NX + GW; ++k)
                for (int j = -GW; j < NX + GW; ++j)
                    for (int ii = -GW; ii < NX + GW; ++ii) {
                        if (ii >= 0 && ii < NX && j >= 0 && j < NX && k >= 0 && k < NX) continue;
                        const int off[3] = {ii, j, k};
                        int64_t g[3];
                        for (int a = 0; a < 3; ++a) g[a] = E * c[a] + to[a] + off[a];
                        fold(l, g);
                        int lc = 0;
                        const int64_t src = entry(l, g, &lc);
                        if (src == INT64_MIN)
                            return fail(nullptr, HYDRO_EINVAL,
                                        "ghost cell of leaf " + std::to_string(i) +
                                            " is neither covered nor refined once (tree not 2:1 balanced)");
                        if (!linear || lc >= l) {
                            m[s++] = (int32_t)src;
                            continue;
                        }
                        if (lc != l - 1)
                            return fail(nullptr, HYDRO_EINVAL, "ghost cell two levels coarser (tree not 2:1 balanced)");
                        // prolongation row: the coarse cell C, its six neighbours
                        // at C's level, and the side of g within C per axis
                        if (rows < capacity && table) {
                            int32_t *r = table + (size_t)rows * PROLONG_ROW;
                            const int64_t C[3] = {g[0] >> 1, g[1] >> 1, g[2] >> 1};
                            int lcc = 0;
                            r[0] = (int32_t)entry(lc, C, &lcc);
                            for (int a = 0; a < 3; ++a)
                                for (int side = 0; side < 2; ++side) {
                                    int64_t q[3] = {C[0], C[1], C[2]};
                                    q[a] += side ? 1 : -1;
                                    fold(lc, q);
                                    const int64_t e = entry(lc, q, &lcc);
                                    if (e == INT64_MIN)
                                        return fail(nullptr, HYDRO_EINVAL, "coarse neighbour not covered (tree not 2:1 balanced)");
                                    r[1 + 2 * a + side] = (int32_t)e;
                                }
                            r[7] = (int32_t)((g[0] & 1) | ((g[1] & 1) << 1) | ((g[2] & 1) << 2));
                        }
                        m[s++] = -PROLONG_BASE - 1 - rows;
                        ++rows;
                    }
        }
    }
    if (linear) {
        *n_table = rows;
        if (rows > capacity) return fail(nullptr, HYDRO_ENOMEM, "prolongation table needs " + std::to_string(rows) + " rows");
    }
    return HYDRO_OK;
}

}  // namespace

// Set-up and error text shared with the allocation-free entry point
// (hydro_noalloc.hip), which has no handle.
hipError_t hydro_internal_ghost_table(int dev) { return ensure_ghost_table(dev); }
void hydro_internal_set_error(const char *msg) { g_create_err = msg; }

// Launcher of the attainable-rate probe (probe_kernels.hip).
hipError_t hydro_launch_fp64_probe(double *out, int blocks, int iters, double m, double c, hipStream_t s);

extern "C" {

int hydro_create(const hydro_params *p, hydro_t **out) {
    if (!out) return fail(nullptr, HYDRO_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(nullptr, HYDRO_EINVAL, "params is NULL");
    if (p->max_leaves <= 0) return fail(nullptr, HYDRO_EINVAL, "max_leaves must be > 0");
    if (p->recon != 0 && p->recon != 1) return fail(nullptr, HYDRO_EINVAL, "recon must be 0 or 1");
    if (p->mlp_batch < 0) return fail(nullptr, HYDRO_EINVAL, "mlp_batch must be >= 0");
    if (p->rk_order != 0 && p->rk_order != 2 && p->rk_order != 3)
        return fail(nullptr, HYDRO_EINVAL, "rk_order must be 2 or 3");
    if (p->scheme != 0 && p->scheme != 1) return fail(nullptr, HYDRO_EINVAL, "scheme must be 0 or 1");
    if (p->reflux != 0 && p->reflux != 1) return fail(nullptr, HYDRO_EINVAL, "reflux must be 0 or 1");
    if (p->leaf_edge != 0 && p->leaf_edge != 8 && p->leaf_edge != 16)
        return fail(nullptr, HYDRO_EINVAL, "leaf_edge must be 8 or 16");
    if ((int64_t)p->max_leaves * (p->leaf_edge == 16 ? 4096 : 512) > INT32_MAX)
        return fail(nullptr, HYDRO_EINVAL, "max_leaves too large for int32 cell ids");
    if (p->schedule < HYDRO_SCHED_AUTO || p->schedule > HYDRO_SCHED_TILED)
        return fail(nullptr, HYDRO_EINVAL, "schedule must be one of HYDRO_SCHED_*");
    if (!(p->eta1 >= 0.0) || !(p->eta2 >= 0.0)) return fail(nullptr, HYDRO_EINVAL, "eta1/eta2 must be >= 0");
    hydro_t *h = new (std::nothrow) hydro_t();
    if (!h) return fail(nullptr, HYDRO_ENOMEM, "handle allocation");
    h->p = *p;
    h->device = p->device;
    h->rk = p->rk_order == 3 ? 3 : 2;
    h->ts = p->leaf_edge == 16 ? 3 : 0;
    h->lg = p->leaf_edge == 16 ? 4 : 3;
    int rc = set_device(h);
    if (rc) { g_create_err = h->err; delete h; return rc; }
    hipError_t e = ensure_ghost_table(h->device);
    if (e != hipSuccess) { rc = hip_fail(h, e, "ghost table upload"); g_create_err = h->err; delete h; return rc; }
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, h->device);
    if (e != hipSuccess) { rc = hip_fail(h, e, "hipGetDeviceProperties"); g_create_err = h->err; delete h; return rc; }
    h->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    h->arch = prop.gcnArchName;
    for (int b = 0; b < HYDRO_NBUCKET; ++b) h->table[b] = HYDRO_SCHED_COLUMN;
    if (p->tune_cache && load_table(h, p->tune_cache) != HYDRO_OK) {
        rc = HYDRO_EINVAL;
        g_create_err = h->err;
        delete h;
        return rc;
    }
    const size_t n = (size_t)p->max_leaves << h->ts;   // in 8^3 blocks
    e = hipMalloc((void **)&h->U1, n * LEAF_STRIDE * sizeof(double));
    if (e == hipSuccess && h->rk == 3) e = hipMalloc((void **)&h->U2, n * LEAF_STRIDE * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&h->dscr, n * 3 * LEAF_STRIDE * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&h->amax, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc((void **)&h->queue, QUEUE_INTS * (1 + NSIDE) * sizeof(int));
    for (int i = 0; i < NSIDE && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&h->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->join_ev[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc((void **)&h->leaf_done, n * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void **)&h->tile_amax, n * 3 * sizeof(double));
    if (e == hipSuccess && p->reflux) e = hipMalloc((void **)&h->bflux, n * BFLUX_STRIDE * sizeof(double));
    if (e == hipSuccess) e = alloc_mlp(h, n);
    if (e == hipSuccess) e = hipMemset(h->queue, 0, QUEUE_INTS * (1 + NSIDE) * sizeof(int));
    if (e == hipSuccess) e = hipMemset(h->leaf_done, 0, n * sizeof(int));
    if (e == hipSuccess) e = hipMalloc((void **)&h->status, sizeof(Status));
    if (e == hipSuccess) e = hipMemset(h->status, 0, sizeof(Status));
    if (e == hipSuccess) e = hipMemset(h->amax, 0, n * sizeof(double));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        rc = (e == hipErrorOutOfMemory) ? fail(h, HYDRO_ENOMEM, "workspace allocation")
                                        : hip_fail(h, e, "workspace allocation");
        g_create_err = h->err;
        hydro_destroy(h);
        return rc;
    }
    *out = h;
    return HYDRO_OK;
}

int hydro_destroy(hydro_t *h) {
    if (!h) return HYDRO_OK;
    (void)hipSetDevice(h->device);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    for (int i = 0; i < NSIDE; ++i) {
        if (h->side[i]) (void)hipStreamDestroy(h->side[i]);
        if (h->join_ev[i]) (void)hipEventDestroy(h->join_ev[i]);
    }
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->U1) (void)hipFree(h->U1);
    if (h->U2) (void)hipFree(h->U2);
    if (h->amax) (void)hipFree(h->amax);
    if (h->dscr) (void)hipFree(h->dscr);
    if (h->queue) (void)hipFree(h->queue);
    if (h->leaf_done) (void)hipFree(h->leaf_done);
    if (h->tile_amax) (void)hipFree(h->tile_amax);
    if (h->bflux) (void)hipFree(h->bflux);
    for (void *b : h->mlp_bufs) (void)hipFree(b);
    if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->status) (void)hipFree(h->status);
    delete h;
    return HYDRO_OK;
}

int hydro_step(hydro_t *h, const hydro_grid *g, double dt, double *amax_out) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U || !aligned8(g->U)) return fail(h, HYDRO_EINVAL, "U is NULL or misaligned");
    if (!(dt >= 0.0) || !isfinite(dt)) return fail(h, HYDRO_EINVAL, "dt must be finite and >= 0");
    if ((rc = set_device(h))) return rc;
    if ((rc = run_stages(h, g, dt, nullptr, true))) return rc;
    if (amax_out) {
        hipStream_t s = (hipStream_t)g->stream;
        const size_t nb = (size_t)g->n << h->ts;
        std::vector<double> blk(nb);
        hipError_t e = hipMemcpyAsync(blk.data(), h->amax, sizeof(double) * nb, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(h, e, "amax copy");
        for (int l = 0; l < g->n; ++l) {
            double m = blk[(size_t)l << h->ts];
            for (int t = 1; t < (1 << h->ts); ++t) m = std::max(m, blk[((size_t)l << h->ts) + t]);
            amax_out[l] = m;
        }
        return read_status(h, s);
    }
    return HYDRO_OK;
}

int hydro_stage(hydro_t *h, const hydro_grid *g, int stage, double dt, const double *Uin,
                const double *Un, double *Uout, double *amax) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (stage < 1 || stage > h->rk) return fail(h, HYDRO_EINVAL, "stage must be 1.." + std::to_string(h->rk));
    if (!Uin || !Uout || (stage >= 2 && !Un)) return fail(h, HYDRO_EINVAL, "null stage buffer");
    if (!aligned8(Uin) || !aligned8(Uout) || (Un && !aligned8(Un)))
        return fail(h, HYDRO_EINVAL, "stage buffers must be 8-byte aligned");
    if (Uin == Uout) return fail(h, HYDRO_EINVAL, "Uout may not alias Uin");
    if (!(dt >= 0.0) || !isfinite(dt)) return fail(h, HYDRO_EINVAL, "dt must be finite and >= 0");
    if ((rc = set_device(h))) return rc;
    if (h->ts == 0) return run_stage(h, g, stage, dt, Uin, stage >= 2 ? Un : Uin, Uout, amax, 0);
    if ((rc = run_stage(h, g, stage, dt, Uin, stage >= 2 ? Un : Uin, Uout, h->amax, 0))) return rc;
    return amax ? leaf_amax(h, g, amax) : HYDRO_OK;
}

int hydro_signal_speed(hydro_t *h, const hydro_grid *g, double *amax) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U || !amax) return fail(h, HYDRO_EINVAL, "null U or amax");
    if ((rc = set_device(h))) return rc;
    if (h->ts == 0) return run_stage(h, g, 0, 0.0, g->U, g->U, nullptr, amax, 0, nullptr, false);
    if ((rc = run_stage(h, g, 0, 0.0, g->U, g->U, nullptr, h->amax, 0, nullptr, false))) return rc;
    return leaf_amax(h, g, amax);
}

int hydro_reconstruct(hydro_t *h, const hydro_grid *g, double *out) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U || !out) return fail(h, HYDRO_EINVAL, "null U or out");
    if (h->ts) return fail(h, HYDRO_EINVAL, "hydro_reconstruct supports 8^3 leaves only");
    if ((rc = set_device(h))) return rc;
    hipError_t e = hydro_launch_reconstruct(g->U, g->ghost_map, g->prolong, g->n_prolong, g->n, out,
                                            (hipStream_t)g->stream);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "reconstruct launch");
}

int hydro_step_dev(hydro_t *h, const hydro_grid *g, double cfl, double *dt_dev) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U || !aligned8(g->U) || !dt_dev) return fail(h, HYDRO_EINVAL, "null U or dt_dev");
    if (!(cfl > 0.0) || !isfinite(cfl)) return fail(h, HYDRO_EINVAL, "cfl must be > 0");
    if ((rc = set_device(h))) return rc;
    return run_step_dev(h, g, cfl, dt_dev, true);
}

int hydro_dt(hydro_t *h, const hydro_grid *g, double cfl, double *dt_dev) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U || !dt_dev) return fail(h, HYDRO_EINVAL, "null U or dt_dev");
    if (!(cfl > 0.0) || !isfinite(cfl)) return fail(h, HYDRO_EINVAL, "cfl must be > 0");
    if ((rc = set_device(h))) return rc;
    if ((rc = run_stage(h, g, 0, 0.0, g->U, g->U, nullptr, h->amax, 0, nullptr, false))) return rc;
    hipError_t e = hydro_launch_dt(g->dx, h->amax, g->n, h->ts, cfl, dt_dev, (hipStream_t)g->stream);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "dt launch");
}

int hydro_graph_capture(hydro_t *h, const hydro_grid *g, double cfl, double *dt_dev, int nsteps) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->stream) return fail(h, HYDRO_EINVAL, "graph capture needs a non-default stream");
    if (!g->U || !dt_dev || nsteps <= 0) return fail(h, HYDRO_EINVAL, "null U/dt_dev or nsteps <= 0");
    if (!(cfl > 0.0) || !isfinite(cfl)) return fail(h, HYDRO_EINVAL, "cfl must be > 0");
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)g->stream;
    if (h->graph_exec) { (void)hipGraphExecDestroy(h->graph_exec); h->graph_exec = nullptr; }
    if (h->graph) { (void)hipGraphDestroy(h->graph); h->graph = nullptr; }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamBeginCapture");
    const int64_t cells0 = h->mlp_cells;   // capture records launches, it runs none
    for (int k = 0; k < nsteps && rc == HYDRO_OK; ++k) rc = run_step_dev(h, g, cfl, dt_dev, false);
    h->graph_mlp_cells = h->mlp_cells - cells0;
    h->mlp_cells = cells0;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (rc) { if (graph) (void)hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return hip_fail(h, e, "hipStreamEndCapture");
    h->graph = graph;
    e = hipGraphInstantiate(&h->graph_exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphInstantiate");
    return HYDRO_OK;
}

int hydro_graph_launch(hydro_t *h, void *stream) {
    if (!h) return HYDRO_EINVAL;
    if (!h->graph_exec) return fail(h, HYDRO_EINVAL, "no graph captured");
    int rc = set_device(h);
    if (rc) return rc;
    hipError_t e = hipGraphLaunch(h->graph_exec, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(h, e, "hipGraphLaunch");
    h->mlp_cells += h->graph_mlp_cells;
    return HYDRO_OK;
}

int hydro_autotune(hydro_t *h, const hydro_grid *g, const char *cache_path, int32_t *table) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U) return fail(h, HYDRO_EINVAL, "null U");
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)g->stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(h, HYDRO_EHIP, "hipEventCreate");
    const int32_t saved_sched = h->p.schedule;
    const bool saved_loaded = h->table_loaded;
    const int32_t saved_multi = h->multi_sched;
    hydro_grid sub = *g;
    sub.n_launch = 0;
    sub.launch_off = nullptr;
    sub.n_reflux = 0;   // timing launches over the first leaves only: no coarse/fine fix-up
    int best_prev = HYDRO_SCHED_COLUMN;
    for (int b = 0; b < HYDRO_NBUCKET && rc == HYDRO_OK; ++b) {
        const int size = 1 << b;
        if (size > g->n) { h->table[b] = best_prev; continue; }
        sub.n = size;
        float best_ms = 1e30f;
        int best = HYDRO_SCHED_COLUMN;
        for (int sc = HYDRO_SCHED_FACE; sc <= HYDRO_SCHED_TILED && rc == HYDRO_OK; ++sc) {
            if (sc == HYDRO_SCHED_FACE && h->p.recon == 1) continue;   // no learned variant (runs the column walk)
            h->p.schedule = sc;
            const int reps = size >= 256 ? 3 : 10;
            rc = run_stage(h, &sub, 1, 0.0, g->U, g->U, h->U1, h->amax, 0, nullptr, false);   // warm
            if (rc) break;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && rc == HYDRO_OK; ++r)
                rc = run_stage(h, &sub, 1, 0.0, g->U, g->U, h->U1, h->amax, 0, nullptr, false);
            (void)hipEventRecord(e1, s);
            float ms = 0.f;
            hipError_t e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) { rc = hip_fail(h, e, "autotune timing"); break; }
            if (ms < best_ms) { best_ms = ms; best = sc; }
        }
        h->table[b] = best;
        best_prev = best;
    }
    // the grid's own partition: its launches run concurrently, where a small
    // launch's latency hides behind the large ones and the chip's total work
    // decides; time whole stages with the per-size table and with each
    // schedule for every launch, in two interleaved rounds (each candidate
    // keeps its faster round, so drift of the chip's clock between
    // candidates does not decide), and keep the fastest
    h->multi_sched = -1;
    h->table_loaded = true;
    if (rc == HYDRO_OK && g->n_launch > 1) {
        hydro_grid part = *g;
        part.n_reflux = 0;
        h->p.schedule = HYDRO_SCHED_AUTO;
        constexpr int NCAND = 5, ROUNDS = 2, REPS = 3;
        const int cand[NCAND] = {-1, HYDRO_SCHED_COLUMN, HYDRO_SCHED_PERSISTENT, HYDRO_SCHED_TILED, MULTI_MERGE};
        float cand_ms[NCAND] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
        for (int round = 0; round < ROUNDS && rc == HYDRO_OK; ++round) {
            for (int ci = 0; ci < NCAND && rc == HYDRO_OK; ++ci) {
                h->multi_sched = cand[ci];
                rc = run_stage(h, &part, 1, 0.0, g->U, g->U, h->U1, h->amax, 0, nullptr, false);   // warm
                if (rc) break;
                (void)hipEventRecord(e0, s);
                for (int r = 0; r < REPS && rc == HYDRO_OK; ++r)
                    rc = run_stage(h, &part, 1, 0.0, g->U, g->U, h->U1, h->amax, 0, nullptr, false);
                (void)hipEventRecord(e1, s);
                float ms = 0.f;
                hipError_t e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) { rc = hip_fail(h, e, "autotune timing"); break; }
                if (ms < cand_ms[ci]) cand_ms[ci] = ms;
            }
        }
        int best = 0;
        for (int ci = 1; ci < NCAND; ++ci)
            if (cand_ms[ci] < cand_ms[best]) best = ci;
        h->multi_sched = cand[best];
    }
    h->p.schedule = saved_sched;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        h->table_loaded = saved_loaded;
        h->multi_sched = saved_multi;
        return rc;
    }
    if (table) memcpy(table, h->table, sizeof(h->table));
    if (cache_path) return save_table(h, cache_path);
    return HYDRO_OK;
}

int hydro_mlp_load(hydro_t *h, const float *params) {
    if (!h) return HYDRO_EINVAL;
    if (!params) return fail(h, HYDRO_EINVAL, "null params");
    int rc = set_device(h);
    if (rc) return rc;
    hipError_t e = hipMemcpy(h->mt.par, params, sizeof(float) * mlp::NPAR, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(h->mt.m, 0, sizeof(float) * mlp::NPAR);
    if (e == hipSuccess) e = hipMemset(h->mt.v, 0, sizeof(float) * mlp::NPAR);
    if (e == hipSuccess) e = hydro_mlp_launch_pack(h->mt, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(h, e, "network load");
    h->adam_t = 0;
    h->mlp_loaded = true;
    return HYDRO_OK;
}

int hydro_mlp_save(hydro_t *h, float *params) {
    if (!h) return HYDRO_EINVAL;
    if (!params) return fail(h, HYDRO_EINVAL, "null params");
    int rc = set_device(h);
    if (rc) return rc;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(params, h->mt.par, sizeof(float) * mlp::NPAR, hipMemcpyDeviceToHost);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "network save");
}

int hydro_mlp_forward(hydro_t *h, const float *X, int B, float *Y, void *stream) {
    if (!h) return HYDRO_EINVAL;
    int rc = check_batch(h, X, B);
    if (rc) return rc;
    if (!Y) return fail(h, HYDRO_EINVAL, "null output");
    if (!h->mlp_loaded) return fail(h, HYDRO_EINVAL, "hydro_mlp_load first");
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hydro_mlp_launch_forward(h->mt, X, B, s);
    if (e == hipSuccess)
        e = hipMemcpy2DAsync(Y, 26 * sizeof(float), h->mt.y, 32 * sizeof(float), 26 * sizeof(float), B,
                             hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "network forward");
}

int hydro_mlp_grad(hydro_t *h, const float *X, const float *T, int B, float *grad, float *loss,
                   void *stream) {
    if (!h) return HYDRO_EINVAL;
    int rc = check_batch(h, X, B);
    if (rc) return rc;
    if (!T || !grad) return fail(h, HYDRO_EINVAL, "null targets or gradient");
    if (!h->mlp_loaded) return fail(h, HYDRO_EINVAL, "hydro_mlp_load first");
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hydro_mlp_launch_forward(h->mt, X, B, s);
    if (e == hipSuccess) e = hydro_mlp_launch_grad(h->mt, T, B, loss, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad, h->mt.grad, sizeof(float) * mlp::NPAR, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "network gradient");
}

int hydro_mlp_train_step(hydro_t *h, const float *X, const float *T, int B, double lr, float *loss,
                         void *stream) {
    if (!h) return HYDRO_EINVAL;
    int rc = check_batch(h, X, B);
    if (rc) return rc;
    if (!T) return fail(h, HYDRO_EINVAL, "null targets");
    if (!(lr > 0.0) || !isfinite(lr)) return fail(h, HYDRO_EINVAL, "lr must be > 0");
    if (!h->mlp_loaded) return fail(h, HYDRO_EINVAL, "hydro_mlp_load first");
    if ((rc = set_device(h))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const double b1 = 0.9, b2 = 0.999;
    ++h->adam_t;
    const float c1 = (float)(1.0 - pow(b1, h->adam_t)), c2 = (float)(1.0 - pow(b2, h->adam_t));
    hipError_t e = hydro_mlp_launch_forward(h->mt, X, B, s);
    if (e == hipSuccess) e = hydro_mlp_launch_grad(h->mt, T, B, loss, s);
    if (e == hipSuccess) e = hydro_mlp_launch_adam(h->mt, (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2, s);
    if (e == hipSuccess) e = hydro_mlp_launch_pack(h->mt, s);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "network train step");
}

int hydro_mlp_pairs(hydro_t *h, const hydro_grid *g, float *X, float *T, uint8_t *valid) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U || !X || !T || !valid) return fail(h, HYDRO_EINVAL, "null U or pair buffer");
    if (h->ts) return fail(h, HYDRO_EINVAL, "hydro_mlp_pairs supports 8^3 leaves only");
    if ((rc = set_device(h))) return rc;
    hipError_t e = hydro_launch_pairs(g->U, g->ghost_map, g->prolong, g->n_prolong, g->n, X, T, valid,
                                      (hipStream_t)g->stream);
    return e == hipSuccess ? HYDRO_OK : hip_fail(h, e, "pairs launch");
}

int hydro_mlp_values(hydro_t *h, const hydro_grid *g, double *val, uint8_t *ok, float *y) {
    int rc = check_grid(h, g);
    if (rc) return rc;
    if (!g->U || !val != !ok) return fail(h, HYDRO_EINVAL, "null U, or only one of val and ok");
    if (!val && !h->mlp_off) return fail(h, HYDRO_EINVAL, "val is NULL and the handle has no learned workspace");
    if (!h->mlp_loaded) return fail(h, HYDRO_EINVAL, "hydro_mlp_load first");
    if ((rc = set_device(h))) return rc;
    mlp::MlpInfer m{};
    m.U = g->U;
    m.gmap = g->ghost_map;
    m.wbi = h->mt.wbi;
    m.bi = h->mt.bi;
    m.val = val;
    m.off = val ? nullptr : h->mlp_off;
    m.alias = val ? nullptr : g->mlp_alias;   // into the workspace: exactly a stage's pre-pass
    m.cell_ok = ok ? ok : h->mlp_ok;
    m.fb_count = h->fb_count;
    m.leaf0 = 0;
    m.ts = h->ts;
    m.lg = h->lg;
    m.prolong = g->prolong;
    m.n_prolong = g->n_prolong;
    m.yraw = y;
    const int nblk = g->n << h->ts;
    hipError_t e = hydro_mlp_launch_infer(m, nblk, (hipStream_t)g->stream);
    if (e != hipSuccess) return hip_fail(h, e, "inference launch");
    h->mlp_cells += (int64_t)nblk * NC;
    return HYDRO_OK;
}

int hydro_mlp_stats(hydro_t *h, int64_t *cells, int64_t *fallback) {
    if (!h) return HYDRO_EINVAL;
    int rc = set_device(h);
    if (rc) return rc;
    unsigned long long fb = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&fb, h->fb_count, sizeof fb, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemset(h->fb_count, 0, sizeof fb);
    if (e != hipSuccess) return hip_fail(h, e, "network statistics");
    if (cells) *cells = h->mlp_cells;
    if (fallback) *fallback = (int64_t)fb;
    h->mlp_cells = 0;
    return HYDRO_OK;
}

const double *hydro_amax_device(const hydro_t *h) { return h ? h->amax : nullptr; }

int hydro_check(hydro_t *h, void *stream) {
    if (!h) return HYDRO_EINVAL;
    int rc = set_device(h);
    if (rc) return rc;
    return read_status(h, (hipStream_t)stream);
}

int hydro_fp64_probe(double *out, int32_t blocks, int32_t iters, double m, double c, void *stream) {
    if (!out || blocks <= 0 || iters < 0) return fail(nullptr, HYDRO_EINVAL, "null out, blocks <= 0 or iters < 0");
    if (((uintptr_t)out & 7u) != 0) return fail(nullptr, HYDRO_EINVAL, "out is misaligned");
    hipError_t e = hydro_launch_fp64_probe(out, blocks, iters, m, c, (hipStream_t)stream);
    return e == hipSuccess ? HYDRO_OK : fail(nullptr, HYDRO_EHIP, std::string("probe launch: ") + hipGetErrorString(e));
}

int hydro_timing(hydro_t *h, int enable, double *total_ms, int64_t *launches) {
    if (!h) return HYDRO_EINVAL;
    int rc = set_device(h);
    if (rc) return rc;
    if (total_ms || launches) {
        double ms = 0.0;
        for (size_t i = 0; i < h->ev_used; ++i) {
            hipError_t e = hipEventSynchronize(h->ev[2 * i + 1]);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, h->ev[2 * i], h->ev[2 * i + 1]);
            if (e != hipSuccess) return hip_fail(h, e, "event timing");
            ms += t;
        }
        if (total_ms) *total_ms = ms;
        if (launches) *launches = (int64_t)h->ev_used;
        h->ev_used = 0;
    }
    if (enable && h->ev.empty()) {
        h->ev.resize(2 * 4096);
        for (auto &e : h->ev) {
            hipError_t err = hipEventCreate(&e);
            if (err != hipSuccess) return hip_fail(h, err, "hipEventCreate");
        }
    }
    h->timing = enable != 0;
    return HYDRO_OK;
}

const char *hydro_strerror(int code) {
    switch (code) {
    case HYDRO_OK: return "ok";
    case HYDRO_EINVAL: return "invalid argument";
    case HYDRO_ENOMEM: return "out of workspace or device memory";
    case HYDRO_EHIP: return "HIP runtime error";
    case HYDRO_ENONPHYS: return "non-physical state";
    default: return "unknown error";
    }
}

const char *hydro_last_error(const hydro_t *h) { return h ? h->err.c_str() : g_create_err.c_str(); }

// ---------------------------------------------------------------------------
// Ghost map of an octree (host)
// ---------------------------------------------------------------------------


int hydro_ghost_map(const hydro_tree *t, int32_t *map) {
    return build_ghost_map(t, map, nullptr, 0, nullptr);
}

int hydro_ghost_map_linear(const hydro_tree *t, int32_t *map, int32_t *table, int32_t capacity,
                           int32_t *n_table) {
    if (!n_table) return fail(nullptr, HYDRO_EINVAL, "null n_table");
    if (capacity < 0) return fail(nullptr, HYDRO_EINVAL, "capacity < 0");
    return build_ghost_map(t, map, table, capacity, n_table);
}

int hydro_mlp_alias_map(const hydro_tree *t, const int32_t *map, int32_t *alias) {
    if (!map || !alias) return fail(nullptr, HYDRO_EINVAL, "null map or alias");
    TreeIndex ti;
    int rc = ti.build(t);   // validates the tree (levels, coordinates, leaf edge)
    if (rc) return rc;
    const int lg = t->leaf_edge == 16 ? 4 : 3;
    const int64_t E = (int64_t)1 << lg, cells = E * E * E;
    const int tiles = t->leaf_edge == 16 ? 8 : 1;
    const int64_t nblk = (int64_t)t->n * tiles;
    const std::vector<int16_t> pg = pad_ghost_table();
    // what fills padded cell (i, j, k) of block b: the global index of an
    // interior cell, or the block's ghost-map entry (a copy, a mean or a
    // prolongation row); equal descriptors mean equal values in any state
    auto desc = [&](int64_t b, int i, int j, int k) -> int64_t {
        if (i >= 0 && i < NX && j >= 0 && j < NX && k >= 0 && k < NX) {
            const int tile = (int)(b % tiles);
            const int64_t x = 8 * (tile & 1) + i, y = 8 * ((tile >> 1) & 1) + j, z = 8 * (tile >> 2) + k;
            return (b / tiles) * cells + (z * E + y) * E + x;
        }
        return map[b * NG + pg[((k + GW) * PB + (j + GW)) * PB + (i + GW)]];
    };
    constexpr int NGS = mlp::NSLOT - NC;   // 384 face-adjacent ghost cells
    for (int64_t b = 0; b < nblk; ++b) {
        for (int s = 0; s < NGS; ++s) {
            const int slab = s / 64, u = s % 8, v = (s / 8) % 8, side = slab & 1;
            const int e = side ? NX : -1;
            const int i = slab < 2 ? e : u, j = slab < 2 ? u : (slab < 4 ? e : v), k = slab < 4 ? v : e;
            int32_t out = -1;
            const int64_t src = desc(b, i, j, k);
            if (src >= 0 && src < (int64_t)t->n * cells) {
                // the copied cell X: interior cell (ci, cj, ck) of block b2
                const int64_t loc = src % cells;
                const int x = (int)(loc % E), y = (int)((loc / E) % E), z = (int)(loc / (E * E));
                const int64_t b2 = (src / cells) * tiles + (((z >> 3) << 2) | ((y >> 3) << 1) | (x >> 3));
                const int ci = x & 7, cj = y & 7, ck = z & 7;
                bool same = true;
                for (int dk = -1; dk <= 1 && same; ++dk)
                    for (int dj = -1; dj <= 1 && same; ++dj)
                        for (int di = -1; di <= 1 && same; ++di)
                            same = desc(b, i + di, j + dj, k + dk) == desc(b2, ci + di, cj + dj, ck + dk);
                if (same) out = (int32_t)(b2 * mlp::NSLOT + (ck * NX + cj) * NX + ci);
            }
            alias[b * NGS + s] = out;
        }
    }
    return HYDRO_OK;
}

int hydro_reflux_map(const hydro_tree *t, int32_t *face_flags, int32_t *entries, int32_t *n_entries) {
    if (!face_flags || !entries || !n_entries) return fail(nullptr, HYDRO_EINVAL, "null output");
    if (t && t->leaf_edge == 16) {
        // a mesh of 16^3 leaves is, cell for cell, the mesh of their 8^3
        // octants (block b = 8 leaf + t at offset 8 (t & 1, t >> 1 & 1, t >> 2)
        // cells, same level on a base grid of twice as many 8^3 leaves), and
        // the kernels work on those blocks: the lists are built there
        if (!t->level || !t->coord) return fail(nullptr, HYDRO_EINVAL, "tree arrays are NULL");
        if (t->n <= 0 || t->n > INT32_MAX / 8) return fail(nullptr, HYDRO_EINVAL, "bad leaf count");
        std::vector<int32_t> lev((size_t)t->n * 8), crd((size_t)t->n * 24);
        for (int i = 0; i < t->n; ++i)
            for (int b = 0; b < 8; ++b) {
                const size_t o = (size_t)i * 8 + b;
                lev[o] = t->level[i];
                crd[3 * o + 0] = 2 * t->coord[3 * (size_t)i + 0] + (b & 1);
                crd[3 * o + 1] = 2 * t->coord[3 * (size_t)i + 1] + ((b >> 1) & 1);
                crd[3 * o + 2] = 2 * t->coord[3 * (size_t)i + 2] + (b >> 2);
            }
        hydro_tree t8 = *t;
        t8.n = t->n * 8;
        for (int a = 0; a < 3; ++a) t8.nb[a] = 2 * t->nb[a];
        t8.level = lev.data();
        t8.coord = crd.data();
        t8.leaf_edge = 8;
        return hydro_reflux_map(&t8, face_flags, entries, n_entries);
    }
    TreeIndex ti;
    int rc = ti.build(t);
    if (rc) return rc;
    for (int i = 0; i < t->n; ++i) face_flags[i] = 0;
    int32_t m = 0;
    for (int i = 0; i < t->n; ++i) {
        const int l = t->level[i];
        const int32_t *c = t->coord + 3 * (size_t)i;
        int32_t *e = entries + (size_t)m * REFLUX_ENTRY;
        int mask = 0;
        for (int k = 0; k < 4 * NBFACE; ++k) e[2 + k] = -1;
        for (int phi = 0; phi < NBFACE; ++phi) {
            const int n = phi >> 1, side = phi & 1;
            int64_t q[3] = {c[0], c[1], c[2]};
            q[n] += side ? 1 : -1;
            const int64_t dim = (int64_t)t->nb[n] << l;
            if (q[n] < 0 || q[n] >= dim) {
                if (t->bc[n] != 0) continue;   // outflow boundary: no neighbour
                q[n] = (q[n] + dim) % dim;
            }
            bool covered = false;   // a leaf of this level or coarser
            for (int lc = l; lc >= 0 && !covered; --lc)
                covered = ti.leaf(lc, q[0] >> (l - lc), q[1] >> (l - lc), q[2] >> (l - lc)) >= 0;
            if (covered) continue;
            const int t1 = (n == 0) ? 1 : 0, t2 = (n == 2) ? 1 : 2;
            for (int o2 = 0; o2 < 2; ++o2)
                for (int o1 = 0; o1 < 2; ++o1) {
                    int64_t r[3];
                    r[n] = 2 * q[n] + (side ? 0 : 1);
                    r[t1] = 2 * q[t1] + o1;
                    r[t2] = 2 * q[t2] + o2;
                    const int32_t ch = ti.leaf(l + 1, r[0], r[1], r[2]);
                    if (ch < 0)
                        return fail(nullptr, HYDRO_EINVAL,
                                    "face " + std::to_string(phi) + " of leaf " + std::to_string(i) +
                                        " is neither covered nor refined once (tree not 2:1 balanced)");
                    e[2 + 4 * phi + o1 + 2 * o2] = ch;
                    face_flags[ch] |= 1 << (8 + 2 * n + (1 - side));
                }
            mask |= 1 << phi;
        }
        if (mask) {
            face_flags[i] |= mask;
            e[0] = i;
            e[1] = mask;
            ++m;
        }
    }
    *n_entries = m;
    return HYDRO_OK;
}

}  // extern "C"
