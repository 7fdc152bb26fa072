// Allocation-free SSP-RK2 step (hydro_step_noalloc in include/hydro.h) for
// callers that cannot allocate device memory: every buffer the step needs
// beyond the caller's inputs and outputs lives in one fixed device array of
// this translation unit, which each GPU holds from library load until the
// process ends.

#include "hydro_common.h"
#include "../../include/hydro.h"

#include <math.h>

#include <atomic>
#include <mutex>
#include <string>

using namespace hydro;

namespace {

constexpr int MAXL = HYDRO_NOALLOC_MAX_LEAVES;
// scratch layout, in doubles: the stage-1 state [MAXL][7][512], the column
// walk's per-axis flux differences [MAXL][3][7][512], per-leaf signal speeds
// [MAXL] (when the caller passes none) and the status word (16 bytes)
constexpr size_t OFF_U1 = 0;
constexpr size_t OFF_W = OFF_U1 + (size_t)MAXL * LEAF_STRIDE;
constexpr size_t OFF_AMAX = OFF_W + (size_t)MAXL * 3 * LEAF_STRIDE;
constexpr size_t OFF_STATUS = OFF_AMAX + MAXL;
constexpr size_t SCRATCH_DOUBLES = OFF_STATUS + 2;
static_assert(sizeof(Status) <= 2 * sizeof(double), "status word must fit its slot");

}  // namespace

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {

constexpr int MAXDEV = 64;
std::once_flag g_once[MAXDEV];
hipError_t g_setup_err[MAXDEV];
double *g_scratch[MAXDEV];   // device address of `scratch` on each device
std::atomic<bool> g_ready[MAXDEV];   // set-up done and succeeded on the device

// Once per device, with that device current: the address of this device's
// copy of the scratch array, and the ghost-slot tables the gather reads.
hipError_t setup(int dev) {
    std::call_once(g_once[dev], [dev] {
        double *p = nullptr;
        hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e == hipSuccess && p == nullptr) e = hipErrorInvalidSymbol;
        if (e == hipSuccess) e = hydro_internal_ghost_table(dev);
        g_scratch[dev] = e == hipSuccess ? p : nullptr;
        g_setup_err[dev] = e;
        g_ready[dev].store(e == hipSuccess, std::memory_order_release);
    });
    return g_setup_err[dev];
}

int fail(int code, const std::string &msg) {
    hydro_internal_set_error(msg.c_str());
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(HYDRO_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// The status word starts each call at zero; a kernel store rather than a
// memset, so that a captured graph holds no memset node.
__global__ void clear_status(Status *s) {
    s->flag = 0;
    s->leaf = 0;
    s->cell = 0;
    s->field = 0;
}

}  // namespace

extern "C" int hydro_step_noalloc(const hydro_grid *g, double dt, double eta1, double eta2, double *amax,
                                  int sync) {
    if (!g) return fail(HYDRO_EINVAL, "grid is NULL");
    if (g->n <= 0) return fail(HYDRO_EINVAL, "grid has no leaves");
    if (g->n > MAXL)
        return fail(HYDRO_EINVAL, "grid has " + std::to_string(g->n) + " leaves; hydro_step_noalloc takes at most " +
                                      std::to_string(MAXL));
    if (!g->U || !g->dx || !g->origin || !g->ghost_map) return fail(HYDRO_EINVAL, "null U/dx/origin/ghost_map");
    if (((uintptr_t)g->U & 7u) != 0) return fail(HYDRO_EINVAL, "U is misaligned");
    if (!(g->gamma > 1.0) || !isfinite(g->gamma)) return fail(HYDRO_EINVAL, "gamma must be > 1");
    if (!isfinite(g->omega)) return fail(HYDRO_EINVAL, "omega must be finite");
    if (!(dt >= 0.0) || !isfinite(dt)) return fail(HYDRO_EINVAL, "dt must be finite and >= 0");
    if (!(eta1 >= 0.0) || !(eta2 >= 0.0) || !isfinite(eta1) || !isfinite(eta2))
        return fail(HYDRO_EINVAL, "eta1/eta2 must be finite and >= 0");
    if (g->face_flags || g->n_reflux) return fail(HYDRO_EINVAL, "hydro_step_noalloc has no flux correction");
    if (g->n_prolong < 0 || (g->n_prolong > 0 && !g->prolong)) return fail(HYDRO_EINVAL, "bad prolongation table");
    if (amax && ((uintptr_t)amax & 7u) != 0) return fail(HYDRO_EINVAL, "amax is misaligned");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= MAXDEV) return fail(HYDRO_EINVAL, "device ordinal out of range");
    hipStream_t s = (hipStream_t)g->stream;
    if (!g_ready[dev].load(std::memory_order_acquire)) {
        // the one-time set-up copies tables to the device: not under capture
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        e = hipStreamIsCapturing(s, &cs);
        if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
        if (cs != hipStreamCaptureStatusNone)
            return fail(HYDRO_EINVAL, "the first hydro_step_noalloc call on a device may not be captured");
        if ((e = setup(dev)) != hipSuccess) return hip_fail(e, "scratch set-up");
    }
    double *const base = g_scratch[dev];
    Status *const status = (Status *)(base + OFF_STATUS);
    hipLaunchKernelGGL(clear_status, dim3(1), dim3(1), 0, s, status);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "status clear");

    StageArgs a{};
    a.dx = g->dx;
    a.origin = g->origin;
    a.gmap = g->ghost_map;
    a.amax = amax ? amax : base + OFF_AMAX;
    a.status = status;
    a.ph = Phys{g->gamma, g->omega, eta1, eta2};
    a.dt = dt;
    a.leaf0 = 0;
    a.nleaf = g->n;
    a.kernel = KERNEL_COLUMN;
    a.tiles = 1;
    a.dscr = base + OFF_W;
    a.ts = 0;
    a.lg = 3;
    a.prolong = g->prolong;
    a.n_prolong = g->n_prolong;
    double *const U1 = base + OFF_U1;
    // stage 1: U1 = U + dt L(U)
    a.stage = 1;
    a.last = 0;
    a.ca = 0.0;
    a.cb = 1.0;
    a.amax_accumulate = 0;
    a.Uin = g->U;
    a.Un = g->U;
    a.Uout = U1;
    if ((e = hydro_launch_stage(a, s)) != hipSuccess) return hip_fail(e, "stage 1 launch");
    // stage 2: U <- U/2 + (U1 + dt L(U1))/2, tracer resync
    a.stage = 2;
    a.last = 1;
    a.ca = 0.5;
    a.cb = 0.5;
    a.amax_accumulate = 1;
    a.Uin = U1;
    a.Un = g->U;
    a.Uout = g->U;
    if ((e = hydro_launch_stage(a, s)) != hipSuccess) return hip_fail(e, "stage 2 launch");
    if (!sync) return HYDRO_OK;
    Status st;
    e = hipMemcpyAsync(&st, status, sizeof st, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "status read");
    if (st.flag) {
        static const char *names[NF] = {"rho", "sx", "sy", "sz", "egas", "tau", "spc"};
        return fail(HYDRO_ENONPHYS, std::string("non-physical ") +
                                        ((st.field >= 0 && st.field < NF) ? names[st.field] : "value") +
                                        " at leaf " + std::to_string(st.leaf) + " cell " + std::to_string(st.cell));
    }
    return HYDRO_OK;
}
