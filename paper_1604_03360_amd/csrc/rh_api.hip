// rh_api.hip -- plan runtime and the exported C ABI (declared in include/rh.h).
//
// A plan describes one grid; the caller owns the state and workspace buffers
// and the stream.  rh_step enqueues, per SSP-RK3 stage (Sec. 1 of Sikorski et
// al., arXiv:1604.03360), one directional sweep per axis longer than one cell,
// in the order x, y, z; the first sweep starts the L accumulator and the last
// one fuses the stage combine.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/rh.h"
#include "rh_internal.hpp"

// Reduction partials of rh_totals_noalloc: [6][kTotalsBlocks] doubles (24 KiB),
// one copy per GPU, held from module load until the process ends.  Host code
// never passes this name to a kernel or a copy (on the host it only stands in
// for the symbol): the device address is looked up once per device with
// hipGetSymbolAddress and that address is used instead.
static __device__ __align__(256) double scratch[6 * rh::kTotalsBlocks];

namespace {

thread_local std::string g_last_error;

rh_status fail(rh_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

rh_status hip_fail(hipError_t e, const char* what) {
    return fail(RH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// roctx range over one library call (host side: enqueue, and the waits of the
// calls that synchronise), visible to rocprofv3 --marker-trace; a push / pop
// pair costs a few tens of nanoseconds when no tool is attached.
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePush(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

// Device address of `scratch` on each device, looked up on the first
// rh_totals_noalloc call made with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

rh_status scratch_for_current_device(double** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RH_E_NOTSUP, "device index beyond the library's table of 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr) return fail(RH_E_HIP, "hipGetSymbolAddress(scratch) gave a null address");
        g_scratch_dev[dev] = (double*)ptr;
    }
    *out = g_scratch_dev[dev];
    return RH_OK;
}

struct TimedLaunch {
    int cls;
    hipEvent_t a, b;
};

}  // namespace

struct rh_plan {
    rh_grid_desc d;
    int ghosts;
    long long ncell;
    size_t elem;                 // bytes per value
    void* state = nullptr;
    void* ws = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    unsigned* d_clamps = nullptr;   // floor counter
    double* d_partials = nullptr;   // [6][kTotalsBlocks]
    double* d_totals = nullptr;     // [6]
    // per-kernel timing
    bool timing = false;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    size_t event_next = 0;
    // evaluation path (RH_PATH_*) and the fused stage's launch shape
    int path = RH_PATH_AUTO;
    int stage_tx = 16;
    int stage_seg = 0;           // 0: default segment for the grid
    // one captured step, replayed by rh_step when enabled
    bool graph_on = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph_n = nullptr;           // kGraphSteps steps in one graph
    hipGraphExec_t graph_exec_n = nullptr;
    double graph_dt = 0.0;
    const void* graph_state = nullptr;
    const void* graph_ws = nullptr;
};

namespace {

hipEvent_t take_event(rh_plan* p) {
    if (p->event_next == p->event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        p->event_pool.push_back(e);
    }
    return p->event_pool[p->event_next++];
}

// Run `launch` (returns hipError_t) bracketed by timing events when enabled.
template <class F>
rh_status timed_launch(rh_plan* p, int cls, F&& launch, const char* what) {
    hipEvent_t a = nullptr, b = nullptr;
    if (p->timing) {
        a = take_event(p);
        b = take_event(p);
        if (!a || !b) return fail(RH_E_HIP, "hipEventCreate failed");
        hipError_t er = hipEventRecord(a, p->stream);
        if (er != hipSuccess) return hip_fail(er, "hipEventRecord");
    }
    hipError_t e = launch();
    if (e != hipSuccess) return hip_fail(e, what);
    if (p->timing) {
        hipError_t er = hipEventRecord(b, p->stream);
        if (er != hipSuccess) return hip_fail(er, "hipEventRecord");
        p->timed.push_back({cls, a, b});
    }
    return RH_OK;
}

template <class T>
rh::SweepArgs<T> base_args(rh_plan* p) {
    rh::SweepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    a.fstride = p->ncell;
    a.n[0] = p->d.nx;
    a.n[1] = p->d.ny;
    a.n[2] = p->d.nz;
    a.eps = (T)(p->d.weno_eps > 0.0 ? p->d.weno_eps : 1e-6);
    a.hb.t0 = p->d.hubble_t0;
    a.hb.e0 = p->d.hubble_e0;
    a.hb.n0 = p->d.hubble_n0;
    a.hb.c0[0] = p->d.x0;
    a.hb.c0[1] = p->d.y0;
    a.hb.c0[2] = p->d.z0;
    a.hb.h[0] = p->d.dx;
    a.hb.h[1] = p->d.dy;
    a.hb.h[2] = p->d.dz;
    a.clamps = p->d_clamps;
    return a;
}

bool any_hubble(const rh_plan* p) {
    return p->d.bc[0] == RH_BC_HUBBLE || p->d.bc[1] == RH_BC_HUBBLE || p->d.bc[2] == RH_BC_HUBBLE;
}

// Grid entry of a fused-stage launch for description d at element offset off.
template <class T>
void fill_stage_grid(rh::StageGrid<T>& g, const rh_grid_desc& d, long long off, int tx, int seg) {
    std::memset(&g, 0, sizeof(g));
    g.off = off;
    g.n[0] = d.nx;
    g.n[1] = d.ny;
    g.n[2] = d.nz;
    const double h[3] = {d.dx, d.dy, d.dz};
    const double c0[3] = {d.x0, d.y0, d.z0};
    for (int a = 0; a < 3; ++a) {
        g.bc[a] = d.bc[a];
        g.inv_h[a] = (T)(1.0 / h[a]);
        g.h[a] = h[a];
        g.c0[a] = c0[a];
    }
    g.eps = (T)(d.weno_eps > 0.0 ? d.weno_eps : 1e-6);
    g.t0 = d.hubble_t0;
    g.e0 = d.hubble_e0;
    g.n0 = d.hubble_n0;
    g.gm1 = d.eos == RH_EOS_IDEAL ? d.eos_gamma - 1.0 : 0.0;
    g.limiter = d.limiter;
    g.mk = d.musta_stages;
    g.lam = (T)d.musta_cfl;
    if (d.scheme == RH_SCHEME_MUSTA) {
        const int n[3] = {d.nx, d.ny, d.nz};
        rh::musta_shape<T>(g, seg > 0 ? seg : rh::musta_default_segment(n));
    } else {
        rh::stage_shape<T>(g, tx, seg);
    }
}

// Descriptions resolved for the kernels: defaults of the optional fields filled in.
void resolve_desc(rh_grid_desc& d) {
    if (d.scheme == RH_SCHEME_MUSTA) {
        if (d.musta_stages == 0) d.musta_stages = 2;
        if (d.musta_cfl == 0.0) d.musta_cfl = 0.9;
    }
    if (d.eos == RH_EOS_IDEAL && d.eos_gamma == 0.0) d.eos_gamma = 5.0 / 3.0;
}

double eos_gm1(const rh_grid_desc& d) { return d.eos == RH_EOS_IDEAL ? d.eos_gamma - 1.0 : 0.0; }

// Features only the fused stage implements: MUSTA-FORCE, local splitting and
// the ideal gas.
bool needs_stage(const rh_grid_desc& d) {
    return d.scheme == RH_SCHEME_MUSTA || d.flux_split == RH_SPLIT_LOCAL || d.eos == RH_EOS_IDEAL;
}

// The adjoint covers the paper's WENO scheme with the conformal fluid and
// global splitting.
bool adjoint_supported(const rh_grid_desc& d) { return !needs_stage(d); }

// Launch one fused-stage evaluation of the scheme of d over nblocks blocks.
template <class T>
hipError_t launch_stage_of(const rh_grid_desc& d, int tx, bool hub, const rh::StageArgs<T>& sa,
                           long long nblocks, hipStream_t s) {
    if (d.scheme == RH_SCHEME_MUSTA) return rh::launch_musta<T>(hub, d.eos, d.limiter, d.musta_stages, sa, nblocks, s);
    return rh::launch_stage<T>(d.scheme, tx, hub, d.flux_split == RH_SPLIT_LOCAL, d.eos, sa, nblocks, s);
}

// The ideal-gas WENO stage reads every cell's velocity, pressure and sound
// speed from a recovery pass run before it (MUSTA-FORCE recovers its own).
bool needs_recovery(const rh_grid_desc& d) { return d.eos == RH_EOS_IDEAL && d.scheme != RH_SCHEME_MUSTA; }

// Path of a single grid's evaluations: the fused stage where it is requested
// or where only it implements the scheme; RH_PATH_AUTO keeps the directional
// sweeps otherwise.
bool use_stage(const rh_plan* p) { return needs_stage(p->d) || p->path == RH_PATH_STAGE; }

// One evaluation of L at time t on `us`; stage == 0 stores L in `lacc`,
// otherwise the stage combine writes `uout` from `us`, `u0` and dt.
template <class T>
rh_status evaluate(rh_plan* p, const T* us, const T* u0, T* lacc, T* uout, double t, double dt,
                   int stage) {
    rh::SweepArgs<T> a = base_args<T>(p);
    a.us = us;
    a.u0 = u0;
    a.lacc = lacc;
    a.uout = uout;
    a.dt = (T)dt;
    a.stage = stage;
    a.hb.t = t;
    const int n[3] = {p->d.nx, p->d.ny, p->d.nz};
    const double h[3] = {p->d.dx, p->d.dy, p->d.dz};
    int active[3], na = 0;
    for (int d = 0; d < 3; ++d)
        if (n[d] > 1) active[na++] = d;
    if (na == 0) {
        if (stage == rh::STAGE_WRITE_L)
            return timed_launch(p, RH_KERNEL_OTHER,
                                [&] { return rh::launch_fill_zero<T>(lacc, 5 * p->ncell, p->stream); },
                                "fill launch");
        return timed_launch(p, RH_KERNEL_OTHER, [&] { return rh::launch_combine<T>(a, p->stream); },
                            "combine launch");
    }
    if (use_stage(p)) {
        rh::StageArgs<T> sa;
        std::memset(&sa, 0, sizeof(sa));
        sa.us = us;
        sa.u0 = u0;
        sa.out = stage == rh::STAGE_WRITE_L ? lacc : uout;
        sa.dt = (T)dt;
        sa.stage = stage;
        sa.t = t;
        sa.clamps = p->d_clamps;
        sa.ngrid = 0;
        const bool musta = p->d.scheme == RH_SCHEME_MUSTA;
        fill_stage_grid<T>(sa.one, p->d, 0, p->stage_tx,
                           p->stage_seg > 0 ? p->stage_seg
                                            : (musta ? rh::musta_default_segment(n)
                                                     : rh::stage_default_segment(n, p->stage_tx)));
        const long long nb = rh::stage_blocks(sa.one);
        if (needs_recovery(p->d)) {
            // the workspace's L slot is free on this path (the stage writes uout or lacc)
            sa.prim = (T*)p->ws + 10 * (size_t)p->ncell;
            rh_status st = timed_launch(p, RH_KERNEL_OTHER, [&] {
                return rh::launch_recover_ideal<T>(sa, rh::recover_blocks(sa.one), p->stream);
            }, "recovery launch");
            if (st != RH_OK) return st;
        }
        return timed_launch(p, RH_KERNEL_STAGE, [&] {
            return launch_stage_of<T>(p->d, p->stage_tx, any_hubble(p), sa, nb, p->stream);
        }, "stage launch");
    }
    int i0 = 0;
    if (na >= 2 && active[0] == 0 && active[1] == 1 && rh::sweep_xy_applies(p->d.scheme, n, p->d.bc[0])) {
        // x and y in one launch
        rh::SweepArgs<T> b = a;
        b.first = 1;
        b.stage = na == 2 ? stage : rh::STAGE_WRITE_L;
        b.bc = p->d.bc[1];
        b.inv_h = (T)(1.0 / h[1]);
        const T inv_hx = (T)(1.0 / h[0]);
        rh_status st = timed_launch(p, RH_KERNEL_SWEEP_XY,
                                    [&] { return rh::launch_sweep_xy<T>(p->d.scheme, b, inv_hx, p->stream); },
                                    "sweep launch");
        if (st != RH_OK) return st;
        i0 = 2;
    }
    for (int i = i0; i < na; ++i) {
        const int d = active[i];
        rh::SweepArgs<T> b = a;
        b.first = i == 0;
        b.stage = i == na - 1 ? stage : rh::STAGE_WRITE_L;
        b.bc = p->d.bc[d];
        b.inv_h = (T)(1.0 / h[d]);
        rh_status st = timed_launch(p, RH_KERNEL_SWEEP_X + d,
                                    [&] { return rh::launch_sweep<T>(d, p->d.scheme, b, p->stream); },
                                    "sweep launch");
        if (st != RH_OK) return st;
    }
    return RH_OK;
}

template <class T>
rh_status one_step(rh_plan* p, double dt, double t, T* stages) {
    const size_t S = 5 * (size_t)p->ncell;
    T* U0 = (T*)p->state;
    T* U1 = stages ? stages : (T*)p->ws;   // stage states go to the caller's store if given
    T* U2 = U1 + S;
    T* Lc = (T*)p->ws + 2 * S;
    rh_status st;
    {
        TraceRange r("rh stage 1");
        st = evaluate<T>(p, U0, U0, Lc, U1, t, dt, rh::STAGE_1);
    }
    if (st == RH_OK) {
        TraceRange r("rh stage 2");
        st = evaluate<T>(p, U1, U0, Lc, U2, t + dt, dt, rh::STAGE_2);
    }
    if (st == RH_OK) {
        TraceRange r("rh stage 3");
        st = evaluate<T>(p, U2, U0, Lc, U0, t + 0.5 * dt, dt, rh::STAGE_3);
    }
    return st;
}

void drop_graph(rh_plan* p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->graph_exec_n) (void)hipGraphExecDestroy(p->graph_exec_n);
    if (p->graph_n) (void)hipGraphDestroy(p->graph_n);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    p->graph_exec_n = nullptr;
    p->graph_n = nullptr;
}

// Steps per replay of the multi-step graph: a graph launch boundary costs about
// 10 us of idle GPU between the last kernel of one replay and the first of the
// next, which a graph of several steps pays once.
constexpr int kGraphSteps = 4;

// Capture `count` steps of size dt into *graph and instantiate them in *exec.
template <class T>
rh_status capture_steps(rh_plan* p, double dt, double t, int count, hipGraph_t* graph, hipGraphExec_t* exec) {
    hipError_t e;
    if (!p->cap_stream && (e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "hipStreamCreateWithFlags");
    if ((e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
    hipStream_t keep = p->stream;
    p->stream = p->cap_stream;
    rh_status st = RH_OK;
    for (int k = 0; k < count && st == RH_OK; ++k) st = one_step<T>(p, dt, t + k * dt, nullptr);
    p->stream = keep;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != RH_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    *graph = g;
    if ((e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0)) != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    return RH_OK;
}

// n steps: eager launches, or replays of captured steps when graphs are on
// (kGraphSteps steps per replay while at least that many remain, then single
// steps; not with analytic boundaries, whose stage times change every step,
// and not while per-launch timing is on)
template <class T>
rh_status step_impl(rh_plan* p, double dt, int nsteps, double t, T* stages = nullptr) {
    const bool use_graph = p->graph_on && !stages && !any_hubble(p) && !p->timing;
    if (!use_graph) {
        for (int s = 0; s < nsteps; ++s) {
            rh_status st = one_step<T>(p, dt, t, stages);
            if (st != RH_OK) return st;
            t += dt;
        }
        return RH_OK;
    }
    if (nsteps == 0) return RH_OK;
    if (!p->graph_exec || p->graph_dt != dt || p->graph_state != p->state || p->graph_ws != p->ws) {
        drop_graph(p);
        rh_status st = capture_steps<T>(p, dt, t, 1, &p->graph, &p->graph_exec);
        if (st != RH_OK) {
            drop_graph(p);
            return st;
        }
        p->graph_dt = dt;
        p->graph_state = p->state;
        p->graph_ws = p->ws;
    }
    if (nsteps >= kGraphSteps && !p->graph_exec_n) {
        rh_status st = capture_steps<T>(p, dt, t, kGraphSteps, &p->graph_n, &p->graph_exec_n);
        if (st != RH_OK) {
            drop_graph(p);
            return st;
        }
    }
    int k = 0;
    for (; k + kGraphSteps <= nsteps; k += kGraphSteps) {
        hipError_t e = hipGraphLaunch(p->graph_exec_n, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    for (; k < nsteps; ++k) {
        hipError_t e = hipGraphLaunch(p->graph_exec, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    return RH_OK;
}

bool is_fp32(const rh_plan* p) { return p->d.precision == RH_PREC_FP32; }

rh_status check_bound(const rh_plan* p) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    if (!p->bound) return fail(RH_E_STATE, "plan has no bound state/workspace (call rh_bind)");
    return RH_OK;
}

}  // namespace

extern "C" {

const char* rh_last_error(void) { return g_last_error.c_str(); }

const char* rh_version(void) { return "rh-mi355x 0.1 (gfx950; WENO5/7, SSP-RK3, FP64/FP32)"; }

rh_status rh_plan_create(rh_plan** out, const rh_grid_desc* d) {
    if (!out) return fail(RH_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!d) return fail(RH_E_INVAL, "grid description is NULL");
    const int n[3] = {d->nx, d->ny, d->nz};
    const double h[3] = {d->dx, d->dy, d->dz};
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 1) return fail(RH_E_INVAL, "cell counts must be >= 1");
        if (!(h[a] > 0.0) || !std::isfinite(h[a])) return fail(RH_E_INVAL, "cell widths must be > 0");
        if (d->bc[a] < RH_BC_PERIODIC || d->bc[a] > RH_BC_HUBBLE)
            return fail(RH_E_INVAL, "unknown boundary condition");
    }
    if (n[0] > (1 << 24) || n[1] > (1 << 24) || n[2] > (1 << 24))
        return fail(RH_E_INVAL, "axis longer than 2^24 cells");
    const bool musta = d->scheme == RH_SCHEME_MUSTA;
    if (d->scheme != 5 && d->scheme != 7 && !musta)
        return fail(RH_E_INVAL, "scheme must be 5, 7 or RH_SCHEME_MUSTA");
    if (d->precision != RH_PREC_FP64 && d->precision != RH_PREC_FP32)
        return fail(RH_E_INVAL, "unknown precision");
    if (d->weno_eps < 0.0) return fail(RH_E_INVAL, "weno_eps must be >= 0");
    if (d->eos != RH_EOS_CONFORMAL && d->eos != RH_EOS_IDEAL) return fail(RH_E_INVAL, "unknown equation of state");
    if (d->eos == RH_EOS_IDEAL && !(d->eos_gamma == 0.0 || (d->eos_gamma > 1.0 && d->eos_gamma <= 2.0)))
        return fail(RH_E_INVAL, "eos_gamma must lie in (1, 2] (0 selects 5/3)");
    if (d->flux_split != RH_SPLIT_GLOBAL && d->flux_split != RH_SPLIT_LOCAL)
        return fail(RH_E_INVAL, "unknown flux splitting");
    if (musta && d->flux_split != RH_SPLIT_GLOBAL)
        return fail(RH_E_INVAL, "flux splitting applies to the WENO schemes only");
    if (musta) {
        if (d->limiter < RH_LIMITER_MINMOD || d->limiter > RH_LIMITER_NONE)
            return fail(RH_E_INVAL, "unknown slope limiter");
        if (d->musta_stages < 0 || d->musta_stages > 8)
            return fail(RH_E_INVAL, "musta_stages must lie in 1..8 (0 selects 2)");
        if (!(d->musta_cfl == 0.0 || (d->musta_cfl > 0.0 && d->musta_cfl <= 1.0)))
            return fail(RH_E_INVAL, "musta_cfl must lie in (0, 1] (0 selects 0.9)");
    }
    const long long ny_nz = (long long)n[1] * n[2];
    if ((ny_nz + 3) / 4 > 65535LL * 64 && n[0] > 1) return fail(RH_E_INVAL, "grid too large");
    if ((long long)(n[1] + 3) / 4 > 65535 || (long long)(n[2] + 3) / 4 > 65535)
        return fail(RH_E_INVAL, "transverse axis too long for the launch grid");
    for (int a = 0; a < 3; ++a) {
        if (d->bc[a] == RH_BC_HUBBLE && !(d->hubble_t0 > 0.0))
            return fail(RH_E_INVAL, "HUBBLE boundaries need hubble_t0 > 0");
        if (d->bc[a] == RH_BC_HUBBLE && d->eos != RH_EOS_CONFORMAL)
            return fail(RH_E_NOTSUP, "HUBBLE boundaries are the conformal fluid's analytic flow");
    }
    // the sweeps address one field with 32-bit byte offsets
    const long long field_bytes = (long long)n[0] * n[1] * n[2] * (d->precision == RH_PREC_FP32 ? 4 : 8);
    if (field_bytes >= (1LL << 32)) return fail(RH_E_INVAL, "one field must be smaller than 4 GiB");
    rh_plan* p = new (std::nothrow) rh_plan();
    if (!p) return fail(RH_E_NOMEM, "host allocation failed");
    p->d = *d;
    resolve_desc(p->d);
    p->ghosts = musta ? 2 : (d->scheme + 1) / 2;
    p->ncell = (long long)n[0] * n[1] * n[2];
    p->elem = d->precision == RH_PREC_FP32 ? 4 : 8;
    hipError_t e;
    if ((e = hipMalloc(&p->d_clamps, sizeof(unsigned))) != hipSuccess ||
        (e = hipMalloc(&p->d_partials, 6 * rh::kTotalsBlocks * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&p->d_totals, 6 * sizeof(double))) != hipSuccess) {
        rh_plan_destroy(p);
        return e == hipErrorOutOfMemory ? fail(RH_E_NOMEM, "hipMalloc failed")
                                        : hip_fail(e, "hipMalloc");
    }
    if ((e = hipMemset(p->d_clamps, 0, sizeof(unsigned))) != hipSuccess) {
        rh_plan_destroy(p);
        return hip_fail(e, "hipMemset");
    }
    *out = p;
    return RH_OK;
}

void rh_plan_destroy(rh_plan* p) {
    if (!p) return;
    if (p->stream) (void)hipStreamSynchronize(p->stream);
    drop_graph(p);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->d_clamps) (void)hipFree(p->d_clamps);
    if (p->d_partials) (void)hipFree(p->d_partials);
    if (p->d_totals) (void)hipFree(p->d_totals);
    for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
    delete p;
}

size_t rh_state_bytes(const rh_plan* p) { return p ? 5 * (size_t)p->ncell * p->elem : 0; }

size_t rh_workspace_bytes(const rh_plan* p) { return p ? 3 * rh_state_bytes(p) : 0; }

rh_status rh_bind(rh_plan* p, void* state, void* workspace, void* stream) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    if (!state || !workspace) return fail(RH_E_INVAL, "state and workspace must be non-NULL");
    if (((uintptr_t)state | (uintptr_t)workspace) & 15)
        return fail(RH_E_INVAL, "buffers must be 16-byte aligned");
    p->state = state;
    p->ws = workspace;
    p->stream = (hipStream_t)stream;
    p->bound = true;
    return RH_OK;
}

rh_status rh_set_fields(rh_plan* p, const double* src, int kind) {
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!src) return fail(RH_E_INVAL, "src is NULL");
    if (kind != RH_FIELDS_CONSERVED && kind != RH_FIELDS_PRIMITIVE) return fail(RH_E_INVAL, "bad kind");
    return timed_launch(p, RH_KERNEL_OTHER, [&] {
        return is_fp32(p) ? rh::launch_set_fields<float>((float*)p->state, src, kind, p->ncell, p->d.eos,
                                                         eos_gm1(p->d), p->stream)
                          : rh::launch_set_fields<double>((double*)p->state, src, kind, p->ncell, p->d.eos,
                                                          eos_gm1(p->d), p->stream);
    }, "set_fields launch");
}

rh_status rh_get_fields(rh_plan* p, double* dst, int kind) {
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!dst) return fail(RH_E_INVAL, "dst is NULL");
    if (kind != RH_FIELDS_CONSERVED && kind != RH_FIELDS_PRIMITIVE) return fail(RH_E_INVAL, "bad kind");
    return timed_launch(p, RH_KERNEL_OTHER, [&] {
        return is_fp32(p) ? rh::launch_get_fields<float>((const float*)p->state, dst, kind, p->ncell,
                                                         p->d_clamps, p->d.eos, eos_gm1(p->d), p->stream)
                          : rh::launch_get_fields<double>((const double*)p->state, dst, kind, p->ncell,
                                                          p->d_clamps, p->d.eos, eos_gm1(p->d), p->stream);
    }, "get_fields launch");
}

rh_status rh_apply_L(rh_plan* p, double t, void* L_out) {
    TraceRange trace("rh_apply_L");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!L_out) return fail(RH_E_INVAL, "L_out is NULL");
    const size_t sb = rh_state_bytes(p);
    const char* lo = (const char*)L_out;
    const char* s0 = (const char*)p->state;
    const char* w0 = (const char*)p->ws;
    if ((lo < s0 + sb && s0 < lo + sb) || (lo < w0 + 3 * sb && w0 < lo + sb))
        return fail(RH_E_INVAL, "L_out aliases the bound buffers");
    if (is_fp32(p))
        return evaluate<float>(p, (const float*)p->state, (const float*)p->state, (float*)L_out,
                               nullptr, t, 0.0, rh::STAGE_WRITE_L);
    return evaluate<double>(p, (const double*)p->state, (const double*)p->state, (double*)L_out,
                            nullptr, t, 0.0, rh::STAGE_WRITE_L);
}

rh_status rh_step(rh_plan* p, double dt, int n_steps, double* t_inout) {
    TraceRange trace("rh_step");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!t_inout) return fail(RH_E_INVAL, "t_inout is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RH_E_INVAL, "dt must be > 0");
    if (n_steps < 0) return fail(RH_E_INVAL, "n_steps must be >= 0");
    st = is_fp32(p) ? step_impl<float>(p, dt, n_steps, *t_inout)
                    : step_impl<double>(p, dt, n_steps, *t_inout);
    if (st == RH_OK) *t_inout += n_steps * dt;
    return st;
}

rh_status rh_set_graph(rh_plan* p, int enable) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    p->graph_on = enable != 0;
    if (!p->graph_on) drop_graph(p);
    return RH_OK;
}

rh_status rh_set_path(rh_plan* p, int path) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    if (path != RH_PATH_AUTO && path != RH_PATH_SWEEPS && path != RH_PATH_STAGE)
        return fail(RH_E_INVAL, "unknown path");
    if (path == RH_PATH_SWEEPS && needs_stage(p->d))
        return fail(RH_E_NOTSUP, "MUSTA-FORCE, local splitting and the ideal gas run on the fused stage only");
    p->path = path;
    drop_graph(p);
    return RH_OK;
}

rh_status rh_get_path(const rh_plan* p, int* path) {
    if (!p || !path) return fail(RH_E_INVAL, "NULL argument");
    *path = use_stage(p) ? RH_PATH_STAGE : RH_PATH_SWEEPS;
    return RH_OK;
}

rh_status rh_set_stage_tuning(rh_plan* p, int tile_x, int seg_z) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    if (tile_x != 16 && tile_x != 32) return fail(RH_E_INVAL, "tile_x must be 16 or 32");
    if (tile_x == 32 && p->d.scheme != 5) return fail(RH_E_NOTSUP, "WENO7 and MUSTA-FORCE stage tiles are 16 cells wide");
    if (seg_z < 0) return fail(RH_E_INVAL, "seg_z must be >= 0 (0 = default)");
    p->stage_tx = tile_x;
    p->stage_seg = seg_z;
    drop_graph(p);
    return RH_OK;
}

rh_status rh_get_stage_tuning(const rh_plan* p, int* tile_x, int* seg_z) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    const int n[3] = {p->d.nx, p->d.ny, p->d.nz};
    if (tile_x) *tile_x = p->stage_tx;
    if (seg_z) *seg_z = p->stage_seg > 0 ? (p->stage_seg < n[2] ? p->stage_seg : n[2])
                                         : (p->d.scheme == RH_SCHEME_MUSTA ? rh::musta_default_segment(n)
                                                                           : rh::stage_default_segment(n, p->stage_tx));
    return RH_OK;
}

rh_status rh_totals(rh_plan* p, double out[5], long long counters[2]) {
    TraceRange trace("rh_totals");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!out) return fail(RH_E_INVAL, "out is NULL");
    st = timed_launch(p, RH_KERNEL_OTHER, [&] {
        return is_fp32(p) ? rh::launch_totals<float>((const float*)p->state, p->ncell, p->d_partials,
                                                     rh::kTotalsBlocks, p->d_totals, p->stream)
                          : rh::launch_totals<double>((const double*)p->state, p->ncell, p->d_partials,
                                                      rh::kTotalsBlocks, p->d_totals, p->stream);
    }, "totals launch");
    if (st != RH_OK) return st;
    double host[6];
    unsigned clamps = 0;
    hipError_t e;
    if ((e = hipMemcpyAsync(host, p->d_totals, sizeof(host), hipMemcpyDeviceToHost, p->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(&clamps, p->d_clamps, sizeof(unsigned), hipMemcpyDeviceToHost, p->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (int f = 0; f < 5; ++f) out[f] = host[f];
    if (counters) {
        counters[0] = clamps;
        counters[1] = (long long)host[5];
    }
    if (p->d.strict && (clamps > 0 || host[5] > 0.0))
        return fail(RH_E_PHYS, "strict plan: a primitive-recovery floor acted or a value is not finite");
    return RH_OK;
}

rh_status rh_totals_integrated(rh_plan* p, double out[5], long long counters[2]) {
    const rh_status st = rh_totals(p, out, counters);
    if (st != RH_OK && st != RH_E_PHYS) return st;
    const double vol = p->d.dx * p->d.dy * p->d.dz;
    for (int f = 0; f < 5; ++f) out[f] *= vol;
    return st;
}

rh_status rh_totals_noalloc(const void* state, int precision, long long ncell, double* out_dev, void* stream) {
    if (!state || !out_dev) return fail(RH_E_INVAL, "state and out_dev must not be NULL");
    if (precision != RH_PREC_FP64 && precision != RH_PREC_FP32) return fail(RH_E_INVAL, "unknown precision");
    const long long elem = precision == RH_PREC_FP32 ? 4 : 8;
    if (ncell < 1 || ncell > (long long)RH_NOALLOC_MAX_BYTES / elem)
        return fail(RH_E_INVAL, "ncell must be >= 1 and one field at most RH_NOALLOC_MAX_BYTES (4 GiB - 1) bytes");
    double* partials = nullptr;
    rh_status st = scratch_for_current_device(&partials);
    if (st != RH_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const hipError_t e =
        precision == RH_PREC_FP32
            ? rh::launch_totals<float>((const float*)state, ncell, partials, rh::kTotalsBlocks, out_dev, s)
            : rh::launch_totals<double>((const double*)state, ncell, partials, rh::kTotalsBlocks, out_dev, s);
    return e == hipSuccess ? RH_OK : hip_fail(e, "totals launch");
}

rh_status rh_reset_counters(rh_plan* p) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    hipError_t e = hipMemsetAsync(p->d_clamps, 0, sizeof(unsigned), p->stream);
    return e == hipSuccess ? RH_OK : hip_fail(e, "hipMemsetAsync");
}

rh_status rh_set_timing(rh_plan* p, int enable) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    if (p->stream || p->bound) (void)hipStreamSynchronize(p->stream);
    p->timing = enable != 0;
    p->timed.clear();
    p->event_next = 0;
    return RH_OK;
}

rh_status rh_kernel_times(rh_plan* p, double* ms_out, long long* launches_out, int n) {
    if (!p) return fail(RH_E_INVAL, "plan is NULL");
    if (n < 0 || n > RH_KERNEL_CLASSES) return fail(RH_E_INVAL, "n out of range");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    std::vector<double> ms(RH_KERNEL_CLASSES, 0.0);
    std::vector<long long> cnt(RH_KERNEL_CLASSES, 0);
    for (const TimedLaunch& t : p->timed) {
        float v = 0.f;
        if ((e = hipEventElapsedTime(&v, t.a, t.b)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        ms[t.cls] += v;
        cnt[t.cls] += 1;
    }
    for (int i = 0; i < n; ++i) {
        if (ms_out) ms_out[i] = ms[i];
        if (launches_out) launches_out[i] = cnt[i];
    }
    return RH_OK;
}

}  // extern "C"

// ===========================================================================
// Event-by-event batches
// ===========================================================================
struct rh_batch {
    std::vector<rh_grid_desc> d;
    std::vector<long long> off;     // ngrid + 1 element offsets
    int ngrid = 0;
    int scheme = 5;
    int precision = RH_PREC_FP64;
    size_t elem = 8;
    bool any_hubble = false;
    // evaluation path and launch shapes
    int path = RH_PATH_AUTO;
    int tile_x = 32, seg[3] = {0, 32, 32};   // directional sweeps
    int nblocks[3] = {0, 0, 0};
    void* d_grids = nullptr;         // BatchGrid<T>[ngrid]
    int stage_tx = 16, stage_seg = 32;       // fused stage
    long long stage_nblocks = 0;
    long long recover_nblocks = 0;   // ideal-gas recovery pass over every grid
    void* d_stage = nullptr;         // StageGrid<T>[ngrid]
    // binding
    void* state = nullptr;
    void* ws = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    unsigned* d_clamps = nullptr;
    double* d_partials = nullptr;
    double* d_totals = nullptr;      // [ngrid][6]
    // graphs
    bool graph_on = false;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    double graph_dt = 0.0;
    const void* graph_state = nullptr;
    const void* graph_ws = nullptr;
    // timing
    bool timing = false;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;
    size_t event_next = 0;
};

namespace {

void drop_graph(rh_batch* b) {
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph_exec = nullptr;
    b->graph = nullptr;
}

template <class T>
rh_status upload_batch_table(rh_batch* b) {
    std::vector<rh::BatchGrid<T>> g(b->ngrid);
    int acc[3] = {0, 0, 0};
    for (int i = 0; i < b->ngrid; ++i) {
        const rh_grid_desc& d = b->d[i];
        rh::BatchGrid<T>& G = g[i];
        std::memset(&G, 0, sizeof(G));
        G.off = b->off[i];
        G.n[0] = d.nx;
        G.n[1] = d.ny;
        G.n[2] = d.nz;
        const double h[3] = {d.dx, d.dy, d.dz};
        const double c0[3] = {d.x0, d.y0, d.z0};
        G.eps = (T)(d.weno_eps > 0.0 ? d.weno_eps : 1e-6);
        G.t0 = d.hubble_t0;
        G.e0 = d.hubble_e0;
        G.n0 = d.hubble_n0;
        for (int a = 0; a < 3; ++a) {
            G.bc[a] = d.bc[a];
            G.inv_h[a] = (T)(1.0 / h[a]);
            G.h[a] = h[a];
            G.c0[a] = c0[a];
            G.seg[a] = b->seg[a] > 0 ? (b->seg[a] < G.n[a] ? b->seg[a] : G.n[a]) : 1;
        }
        int blocks[3];
        rh::batch_blocks(G.n, b->tile_x, G.seg, blocks, G.nchunk);
        for (int c = 0; c < 3; ++c) {
            G.blk0[c] = acc[c];
            acc[c] += blocks[c];
        }
    }
    for (int c = 0; c < 3; ++c) b->nblocks[c] = acc[c];
    if (!b->d_grids) {
        hipError_t e = hipMalloc(&b->d_grids, g.size() * sizeof(rh::BatchGrid<T>));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    }
    hipError_t e = hipMemcpy(b->d_grids, g.data(), g.size() * sizeof(rh::BatchGrid<T>),
                             hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    // fused-stage table: grids in order, each a contiguous range of logical blocks
    std::vector<rh::StageGrid<T>> sg(b->ngrid);
    long long sacc = 0, racc = 0;
    for (int i = 0; i < b->ngrid; ++i) {
        fill_stage_grid<T>(sg[i], b->d[i], b->off[i], b->stage_tx, b->stage_seg);
        sg[i].blk0 = (int)sacc;
        sg[i].rblk0 = (int)racc;
        sacc += rh::stage_blocks(sg[i]);
        racc += rh::recover_blocks(sg[i]);
        if (sacc > 0x7fffffffLL || racc > 0x7fffffffLL)
            return fail(RH_E_NOTSUP, "batch too large for one fused-stage launch");
    }
    b->stage_nblocks = sacc;
    b->recover_nblocks = racc;
    if (!b->d_stage) {
        e = hipMalloc(&b->d_stage, sg.size() * sizeof(rh::StageGrid<T>));
        if (e != hipSuccess) return hip_fail(e, "hipMalloc");
    }
    e = hipMemcpy(b->d_stage, sg.data(), sg.size() * sizeof(rh::StageGrid<T>), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
    drop_graph(b);
    return RH_OK;
}

rh_status upload_table(rh_batch* b) {
    return b->precision == RH_PREC_FP32 ? upload_batch_table<float>(b) : upload_batch_table<double>(b);
}

template <class F>
rh_status batch_timed(rh_batch* b, hipStream_t s, int cls, F&& launch, const char* what) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->timing) {
        for (hipEvent_t* e : {&e0, &e1}) {
            if (b->event_next == b->event_pool.size()) {
                hipEvent_t ev;
                if (hipEventCreate(&ev) != hipSuccess) return fail(RH_E_HIP, "hipEventCreate failed");
                b->event_pool.push_back(ev);
            }
            *e = b->event_pool[b->event_next++];
        }
        hipError_t er = hipEventRecord(e0, s);
        if (er != hipSuccess) return hip_fail(er, "hipEventRecord");
    }
    hipError_t e = launch();
    if (e != hipSuccess) return hip_fail(e, what);
    if (b->timing) {
        hipError_t er = hipEventRecord(e1, s);
        if (er != hipSuccess) return hip_fail(er, "hipEventRecord");
        b->timed.push_back({cls, e0, e1});
    }
    return RH_OK;
}

// One evaluation of L for every grid: three launches (x, y, z), the last one
// fusing the stage combine (stage > 0) or storing L (stage == 0).
template <class T>
rh_status batch_evaluate(rh_batch* b, hipStream_t s, const T* us, const T* u0, T* lacc, T* uout,
                         double t, double dt, int stage, T* prim) {
    if (b->path != RH_PATH_SWEEPS) {
        // one launch: L along x, y and z of every grid and the stage combine
        rh::StageArgs<T> sa;
        std::memset(&sa, 0, sizeof(sa));
        sa.us = us;
        sa.u0 = u0;
        sa.out = stage == rh::STAGE_WRITE_L ? lacc : uout;
        sa.dt = (T)dt;
        sa.stage = stage;
        sa.t = t;
        sa.clamps = b->d_clamps;
        sa.grids = (const rh::StageGrid<T>*)b->d_stage;
        sa.ngrid = b->ngrid;
        if (needs_recovery(b->d[0])) {
            sa.prim = prim;
            rh_status st = batch_timed(b, s, RH_KERNEL_OTHER, [&] {
                return rh::launch_recover_ideal<T>(sa, b->recover_nblocks, s);
            }, "batched recovery launch");
            if (st != RH_OK) return st;
        }
        return batch_timed(b, s, RH_KERNEL_STAGE, [&] {
            return launch_stage_of<T>(b->d[0], b->stage_tx, b->any_hubble, sa, b->stage_nblocks, s);
        }, "batched stage launch");
    }
    rh::BatchArgs<T> B;
    std::memset(&B, 0, sizeof(B));
    B.grids = (const rh::BatchGrid<T>*)b->d_grids;
    B.ngrid = b->ngrid;
    B.base.us = us;
    B.base.u0 = u0;
    B.base.lacc = lacc;
    B.base.uout = uout;
    B.base.dt = (T)dt;
    B.base.hb.t = t;   // epsilon and the analytic-boundary parameters come per grid
    B.base.clamps = b->d_clamps;
    for (int d = 0; d < 3; ++d) {
        rh::BatchArgs<T> Bd = B;
        Bd.base.first = d == 0;
        Bd.base.stage = d == 2 ? stage : rh::STAGE_WRITE_L;
        rh_status st = batch_timed(b, s, RH_KERNEL_SWEEP_X + d, [&] {
            return rh::launch_sweep_batch<T>(d, b->scheme, b->tile_x, Bd, b->nblocks[d], s);
        }, "batched sweep launch");
        if (st != RH_OK) return st;
    }
    return RH_OK;
}

template <class T>
rh_status batch_one_step(rh_batch* b, hipStream_t s, double t, double dt) {
    const size_t S = (size_t)b->off[b->ngrid];
    T* U0 = (T*)b->state;
    T* U1 = (T*)b->ws;
    T* U2 = U1 + S;
    T* Lc = U2 + S;
    // the stage path leaves Lc unused: the ideal gas's recovered fields go there
    rh_status st;
    {
        TraceRange r("rh batch stage 1");
        st = batch_evaluate<T>(b, s, U0, U0, Lc, U1, t, dt, rh::STAGE_1, Lc);
    }
    if (st == RH_OK) {
        TraceRange r("rh batch stage 2");
        st = batch_evaluate<T>(b, s, U1, U0, Lc, U2, t + dt, dt, rh::STAGE_2, Lc);
    }
    if (st == RH_OK) {
        TraceRange r("rh batch stage 3");
        st = batch_evaluate<T>(b, s, U2, U0, Lc, U0, t + 0.5 * dt, dt, rh::STAGE_3, Lc);
    }
    return st;
}

template <class T>
rh_status batch_step_impl(rh_batch* b, double dt, int nsteps, double t) {
    const bool use_graph = b->graph_on && !b->any_hubble && !b->timing;
    if (!use_graph) {
        for (int k = 0; k < nsteps; ++k) {
            rh_status st = batch_one_step<T>(b, b->stream, t, dt);
            if (st != RH_OK) return st;
            t += dt;
        }
        return RH_OK;
    }
    if (!b->graph_exec || b->graph_dt != dt || b->graph_state != b->state || b->graph_ws != b->ws) {
        drop_graph(b);
        hipError_t e;
        if (!b->cap_stream &&
            (e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
            return hip_fail(e, "hipStreamCreateWithFlags");
        if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return hip_fail(e, "hipStreamBeginCapture");
        rh_status st = batch_one_step<T>(b, b->cap_stream, t, dt);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(b->cap_stream, &g);
        if (st != RH_OK) {
            if (g) (void)hipGraphDestroy(g);
            return st;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
        b->graph = g;
        if ((e = hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0)) != hipSuccess) {
            drop_graph(b);
            return hip_fail(e, "hipGraphInstantiate");
        }
        b->graph_dt = dt;
        b->graph_state = b->state;
        b->graph_ws = b->ws;
    }
    for (int k = 0; k < nsteps; ++k) {
        hipError_t e = hipGraphLaunch(b->graph_exec, b->stream);
        if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    }
    return RH_OK;
}

rh_status check_batch(const rh_batch* b) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (!b->bound) return fail(RH_E_STATE, "batch has no bound state/workspace (call rh_batch_bind)");
    return RH_OK;
}

}  // namespace

extern "C" {

rh_status rh_batch_create(rh_batch** out, int n_grids, const rh_grid_desc* descs) {
    if (!out) return fail(RH_E_INVAL, "out is NULL");
    *out = nullptr;
    if (n_grids < 1 || !descs) return fail(RH_E_INVAL, "need at least one grid description");
    rh_batch* b = new (std::nothrow) rh_batch();
    if (!b) return fail(RH_E_NOMEM, "host allocation failed");
    b->ngrid = n_grids;
    b->scheme = descs[0].scheme;
    b->precision = descs[0].precision;
    b->elem = b->precision == RH_PREC_FP32 ? 4 : 8;
    b->off.assign(n_grids + 1, 0);
    long long acc = 0;
    for (int i = 0; i < n_grids; ++i) {
        const rh_grid_desc& d = descs[i];
        // validate each description exactly as a single-grid plan would
        rh_plan* probe = nullptr;
        rh_status st = rh_plan_create(&probe, &d);
        if (st != RH_OK) {
            delete b;
            return st;
        }
        rh_plan_destroy(probe);
        rh_grid_desc r = d, r0 = descs[0];
        resolve_desc(r);
        resolve_desc(r0);
        if (r.scheme != r0.scheme || r.precision != r0.precision || r.eos != r0.eos ||
            (r.eos == RH_EOS_IDEAL && r.eos_gamma != r0.eos_gamma) || r.flux_split != r0.flux_split ||
            (r.scheme == RH_SCHEME_MUSTA && (r.limiter != r0.limiter || r.musta_stages != r0.musta_stages ||
                                             r.musta_cfl != r0.musta_cfl))) {
            delete b;
            return fail(RH_E_INVAL, "all grids of a batch must share scheme, precision, equation of state, "
                                    "flux splitting and the MUSTA-FORCE parameters");
        }
        if (d.nx < 2 || d.ny < 2 || d.nz < 2) {
            delete b;
            return fail(RH_E_NOTSUP, "batched grids need at least 2 cells on every axis");
        }
        for (int a = 0; a < 3; ++a)
            if (d.bc[a] == RH_BC_HUBBLE) b->any_hubble = true;
        b->d.push_back(r);
        b->off[i] = acc;
        const long long n = 5LL * d.nx * d.ny * d.nz;
        acc += (n + 63) / 64 * 64;
    }
    b->off[n_grids] = acc;
    // default launch shape: the x tile that stages the fewest cells over the
    // whole ensemble, 32-cell rolling segments
    long long best = -1;
    for (int tx : {64, 32, 16}) {
        long long staged = 0;
        for (const rh_grid_desc& d : b->d)
            staged += (long long)((d.nx + tx - 1) / tx) * (tx + 2 * ((b->scheme + 1) / 2)) * d.ny * d.nz;
        if (best < 0 || staged < best) {
            best = staged;
            b->tile_x = tx;
        }
    }
    hipError_t e;
    if ((e = hipMalloc(&b->d_clamps, sizeof(unsigned))) != hipSuccess ||
        (e = hipMalloc(&b->d_partials, 6 * rh::kTotalsBlocks * sizeof(double))) != hipSuccess ||
        (e = hipMalloc(&b->d_totals, 6 * (size_t)n_grids * sizeof(double))) != hipSuccess ||
        (e = hipMemset(b->d_clamps, 0, sizeof(unsigned))) != hipSuccess) {
        rh_batch_destroy(b);
        return e == hipErrorOutOfMemory ? fail(RH_E_NOMEM, "hipMalloc failed") : hip_fail(e, "hipMalloc");
    }
    rh_status st = upload_table(b);
    if (st != RH_OK) {
        rh_batch_destroy(b);
        return st;
    }
    *out = b;
    return RH_OK;
}

void rh_batch_destroy(rh_batch* b) {
    if (!b) return;
    drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->d_grids) (void)hipFree(b->d_grids);
    if (b->d_stage) (void)hipFree(b->d_stage);
    if (b->d_clamps) (void)hipFree(b->d_clamps);
    if (b->d_partials) (void)hipFree(b->d_partials);
    if (b->d_totals) (void)hipFree(b->d_totals);
    for (hipEvent_t e : b->event_pool) (void)hipEventDestroy(e);
    delete b;
}

rh_status rh_batch_offsets(const rh_batch* b, long long* offsets) {
    if (!b || !offsets) return fail(RH_E_INVAL, "NULL argument");
    for (int i = 0; i <= b->ngrid; ++i) offsets[i] = b->off[i];
    return RH_OK;
}

size_t rh_batch_state_bytes(const rh_batch* b) { return b ? (size_t)b->off[b->ngrid] * b->elem : 0; }

size_t rh_batch_workspace_bytes(const rh_batch* b) { return b ? 3 * rh_batch_state_bytes(b) : 0; }

rh_status rh_batch_bind(rh_batch* b, void* state, void* workspace, void* stream) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (!state || !workspace) return fail(RH_E_INVAL, "state and workspace must be non-NULL");
    if (((uintptr_t)state | (uintptr_t)workspace) & 15)
        return fail(RH_E_INVAL, "buffers must be 16-byte aligned");
    b->state = state;
    b->ws = workspace;
    b->stream = (hipStream_t)stream;
    b->bound = true;
    return RH_OK;
}

rh_status rh_batch_set_fields(rh_batch* b, const double* src, int kind) {
    rh_status st = check_batch(b);
    if (st != RH_OK) return st;
    if (!src) return fail(RH_E_INVAL, "src is NULL");
    if (kind != RH_FIELDS_CONSERVED && kind != RH_FIELDS_PRIMITIVE) return fail(RH_E_INVAL, "bad kind");
    for (int i = 0; i < b->ngrid; ++i) {
        const long long n = (long long)b->d[i].nx * b->d[i].ny * b->d[i].nz;
        hipError_t e = b->precision == RH_PREC_FP32
            ? rh::launch_set_fields<float>((float*)b->state + b->off[i], src + b->off[i], kind, n, b->d[i].eos,
                                           eos_gm1(b->d[i]), b->stream)
            : rh::launch_set_fields<double>((double*)b->state + b->off[i], src + b->off[i], kind, n, b->d[i].eos,
                                            eos_gm1(b->d[i]), b->stream);
        if (e != hipSuccess) return hip_fail(e, "set_fields launch");
    }
    return RH_OK;
}

rh_status rh_batch_get_fields(rh_batch* b, double* dst, int kind) {
    rh_status st = check_batch(b);
    if (st != RH_OK) return st;
    if (!dst) return fail(RH_E_INVAL, "dst is NULL");
    if (kind != RH_FIELDS_CONSERVED && kind != RH_FIELDS_PRIMITIVE) return fail(RH_E_INVAL, "bad kind");
    for (int i = 0; i < b->ngrid; ++i) {
        const long long n = (long long)b->d[i].nx * b->d[i].ny * b->d[i].nz;
        hipError_t e = b->precision == RH_PREC_FP32
            ? rh::launch_get_fields<float>((const float*)b->state + b->off[i], dst + b->off[i], kind, n,
                                           b->d_clamps, b->d[i].eos, eos_gm1(b->d[i]), b->stream)
            : rh::launch_get_fields<double>((const double*)b->state + b->off[i], dst + b->off[i], kind, n,
                                            b->d_clamps, b->d[i].eos, eos_gm1(b->d[i]), b->stream);
        if (e != hipSuccess) return hip_fail(e, "get_fields launch");
    }
    return RH_OK;
}

rh_status rh_batch_step(rh_batch* b, double dt, int n_steps, double* t_inout) {
    TraceRange trace("rh_batch_step");
    rh_status st = check_batch(b);
    if (st != RH_OK) return st;
    if (!t_inout) return fail(RH_E_INVAL, "t_inout is NULL");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RH_E_INVAL, "dt must be > 0");
    if (n_steps < 0) return fail(RH_E_INVAL, "n_steps must be >= 0");
    st = b->precision == RH_PREC_FP32 ? batch_step_impl<float>(b, dt, n_steps, *t_inout)
                                      : batch_step_impl<double>(b, dt, n_steps, *t_inout);
    if (st == RH_OK) *t_inout += n_steps * dt;
    return st;
}

rh_status rh_batch_totals(rh_batch* b, double* out, long long counters[2]) {
    TraceRange trace("rh_batch_totals");
    rh_status st = check_batch(b);
    if (st != RH_OK) return st;
    if (!out) return fail(RH_E_INVAL, "out is NULL");
    for (int i = 0; i < b->ngrid; ++i) {
        const long long n = (long long)b->d[i].nx * b->d[i].ny * b->d[i].nz;
        hipError_t e = b->precision == RH_PREC_FP32
            ? rh::launch_totals<float>((const float*)b->state + b->off[i], n, b->d_partials,
                                       rh::kTotalsBlocks, b->d_totals + 6 * i, b->stream)
            : rh::launch_totals<double>((const double*)b->state + b->off[i], n, b->d_partials,
                                        rh::kTotalsBlocks, b->d_totals + 6 * i, b->stream);
        if (e != hipSuccess) return hip_fail(e, "totals launch");
    }
    std::vector<double> host(6 * (size_t)b->ngrid);
    unsigned clamps = 0;
    hipError_t e;
    if ((e = hipMemcpyAsync(host.data(), b->d_totals, host.size() * sizeof(double), hipMemcpyDeviceToHost,
                            b->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipMemcpyAsync(&clamps, b->d_clamps, sizeof(unsigned), hipMemcpyDeviceToHost, b->stream)) != hipSuccess)
        return hip_fail(e, "hipMemcpyAsync");
    if ((e = hipStreamSynchronize(b->stream)) != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    double bad = 0.0;
    for (int i = 0; i < b->ngrid; ++i) {
        for (int f = 0; f < 5; ++f) out[5 * i + f] = host[6 * i + f];
        bad += host[6 * i + 5];
    }
    if (counters) {
        counters[0] = clamps;
        counters[1] = (long long)bad;
    }
    bool strict = false;
    for (const rh_grid_desc& d : b->d) strict |= d.strict != 0;
    if (strict && (clamps > 0 || bad > 0.0))
        return fail(RH_E_PHYS, "strict batch: a primitive-recovery floor acted or a value is not finite");
    return RH_OK;
}

rh_status rh_batch_totals_integrated(rh_batch* b, double* out, long long counters[2]) {
    const rh_status st = rh_batch_totals(b, out, counters);
    if (st != RH_OK && st != RH_E_PHYS) return st;
    for (int i = 0; i < b->ngrid; ++i) {
        const double vol = b->d[i].dx * b->d[i].dy * b->d[i].dz;
        for (int f = 0; f < 5; ++f) out[5 * i + f] *= vol;
    }
    return st;
}

rh_status rh_batch_set_graph(rh_batch* b, int enable) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    b->graph_on = enable != 0;
    if (!b->graph_on) drop_graph(b);
    return RH_OK;
}

rh_status rh_batch_set_tuning(rh_batch* b, int tile_x, int seg_y, int seg_z) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (tile_x != 64 && tile_x != 32 && tile_x != 16) return fail(RH_E_INVAL, "tile_x must be 64, 32 or 16");
    if (seg_y < 4 || seg_z < 4) return fail(RH_E_INVAL, "segments must be >= 4 cells");
    b->tile_x = tile_x;
    b->seg[1] = seg_y;
    b->seg[2] = seg_z;
    return upload_table(b);
}

rh_status rh_batch_set_path(rh_batch* b, int path) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (path != RH_PATH_AUTO && path != RH_PATH_SWEEPS && path != RH_PATH_STAGE)
        return fail(RH_E_INVAL, "unknown path");
    if (path == RH_PATH_SWEEPS && needs_stage(b->d[0]))
        return fail(RH_E_NOTSUP, "MUSTA-FORCE, local splitting and the ideal gas run on the fused stage only");
    b->path = path;
    drop_graph(b);
    return RH_OK;
}

rh_status rh_batch_get_path(const rh_batch* b, int* path) {
    if (!b || !path) return fail(RH_E_INVAL, "NULL argument");
    *path = b->path == RH_PATH_SWEEPS ? RH_PATH_SWEEPS : RH_PATH_STAGE;
    return RH_OK;
}

rh_status rh_batch_set_stage_tuning(rh_batch* b, int tile_x, int seg_z) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (tile_x != 16 && tile_x != 32) return fail(RH_E_INVAL, "tile_x must be 16 or 32");
    if (tile_x == 32 && b->scheme != 5) return fail(RH_E_NOTSUP, "WENO7 and MUSTA-FORCE stage tiles are 16 cells wide");
    if (seg_z < 1) return fail(RH_E_INVAL, "seg_z must be >= 1");
    b->stage_tx = tile_x;
    b->stage_seg = seg_z;
    return upload_table(b);
}

rh_status rh_batch_get_stage_tuning(const rh_batch* b, int* tile_x, int* seg_z) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (tile_x) *tile_x = b->stage_tx;
    if (seg_z) *seg_z = b->stage_seg;
    return RH_OK;
}

rh_status rh_batch_get_tuning(const rh_batch* b, int* tile_x, int* seg_y, int* seg_z) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (tile_x) *tile_x = b->tile_x;
    if (seg_y) *seg_y = b->seg[1];
    if (seg_z) *seg_z = b->seg[2];
    return RH_OK;
}

rh_status rh_batch_autotune(rh_batch* b, int reps) {
    TraceRange trace("rh_batch_autotune");
    rh_status st = check_batch(b);
    if (st != RH_OK) return st;
    if (reps < 1) return fail(RH_E_INVAL, "reps must be >= 1");
    hipError_t e;
    hipEvent_t e0, e1;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    const bool saved_timing = b->timing;
    b->timing = false;
    const size_t S = (size_t)b->off[b->ngrid];
    // time one sweep class (evaluations of L into the workspace's accumulator)
    auto time_class = [&](int cls, float* ms) -> rh_status {
        auto one = [&]() -> rh_status {
            if (b->precision == RH_PREC_FP32) {
                float* L = (float*)b->ws + 2 * S;
                rh::BatchArgs<float> B;
                std::memset(&B, 0, sizeof(B));
                B.grids = (const rh::BatchGrid<float>*)b->d_grids;
                B.ngrid = b->ngrid;
                B.base.us = (const float*)b->state;
                B.base.u0 = (const float*)b->state;
                B.base.lacc = L;
                B.base.clamps = b->d_clamps;
                B.base.first = 1;
                B.base.stage = rh::STAGE_WRITE_L;
                hipError_t er = rh::launch_sweep_batch<float>(cls, b->scheme, b->tile_x, B, b->nblocks[cls], b->stream);
                return er == hipSuccess ? RH_OK : hip_fail(er, "autotune launch");
            }
            double* L = (double*)b->ws + 2 * S;
            rh::BatchArgs<double> B;
            std::memset(&B, 0, sizeof(B));
            B.grids = (const rh::BatchGrid<double>*)b->d_grids;
            B.ngrid = b->ngrid;
            B.base.us = (const double*)b->state;
            B.base.u0 = (const double*)b->state;
            B.base.lacc = L;
            B.base.clamps = b->d_clamps;
            B.base.first = 1;
            B.base.stage = rh::STAGE_WRITE_L;
            hipError_t er = rh::launch_sweep_batch<double>(cls, b->scheme, b->tile_x, B, b->nblocks[cls], b->stream);
            return er == hipSuccess ? RH_OK : hip_fail(er, "autotune launch");
        };
        rh_status s2 = one();   // warm-up
        if (s2 != RH_OK) return s2;
        if ((e = hipEventRecord(e0, b->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        for (int r = 0; r < reps; ++r)
            if ((s2 = one()) != RH_OK) return s2;
        if ((e = hipEventRecord(e1, b->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        if ((e = hipEventElapsedTime(ms, e0, e1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        return RH_OK;
    };
    if (b->path != RH_PATH_SWEEPS) {
        // fused stage: x-y tile width and z segment, timed on evaluations of L
        // into the workspace's last state (the ideal gas's recovered fields, in
        // the first, computed once before the timed launches)
        auto time_stage = [&](float* ms) -> rh_status {
            auto one = [&](bool recover) -> rh_status {
                hipError_t er;
                if (b->precision == RH_PREC_FP32) {
                    rh::StageArgs<float> sa;
                    std::memset(&sa, 0, sizeof(sa));
                    sa.us = (const float*)b->state;
                    sa.u0 = (const float*)b->state;
                    sa.out = (float*)b->ws + 2 * S;
                    sa.prim = (float*)b->ws;
                    sa.stage = rh::STAGE_WRITE_L;
                    sa.clamps = b->d_clamps;
                    sa.grids = (const rh::StageGrid<float>*)b->d_stage;
                    sa.ngrid = b->ngrid;
                    if (recover) er = rh::launch_recover_ideal<float>(sa, b->recover_nblocks, b->stream);
                    else er = launch_stage_of<float>(b->d[0], b->stage_tx, b->any_hubble, sa, b->stage_nblocks, b->stream);
                } else {
                    rh::StageArgs<double> sa;
                    std::memset(&sa, 0, sizeof(sa));
                    sa.us = (const double*)b->state;
                    sa.u0 = (const double*)b->state;
                    sa.out = (double*)b->ws + 2 * S;
                    sa.prim = (double*)b->ws;
                    sa.stage = rh::STAGE_WRITE_L;
                    sa.clamps = b->d_clamps;
                    sa.grids = (const rh::StageGrid<double>*)b->d_stage;
                    sa.ngrid = b->ngrid;
                    if (recover) er = rh::launch_recover_ideal<double>(sa, b->recover_nblocks, b->stream);
                    else er = launch_stage_of<double>(b->d[0], b->stage_tx, b->any_hubble, sa, b->stage_nblocks, b->stream);
                }
                return er == hipSuccess ? RH_OK : hip_fail(er, "autotune launch");
            };
            rh_status s2 = needs_recovery(b->d[0]) ? one(true) : RH_OK;
            if (s2 == RH_OK) s2 = one(false);   // warm-up
            if (s2 != RH_OK) return s2;
            if ((e = hipEventRecord(e0, b->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            for (int r = 0; r < reps; ++r)
                if ((s2 = one(false)) != RH_OK) return s2;
            if ((e = hipEventRecord(e1, b->stream)) != hipSuccess) return hip_fail(e, "hipEventRecord");
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
            if ((e = hipEventElapsedTime(ms, e0, e1)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
            return RH_OK;
        };
        int btx = b->stage_tx, bseg = b->stage_seg;
        float bms = 1e30f;
        rh_status rs = RH_OK;
        for (int tx : {16, 32}) {
            if (tx == 32 && b->scheme != 5) continue;
            for (int sg : {16, 24, 32, 48, 64}) {
                b->stage_tx = tx;
                b->stage_seg = sg;
                if ((rs = upload_table(b)) != RH_OK) break;
                float ms;
                if ((rs = time_stage(&ms)) != RH_OK) break;
                if (ms < bms) {
                    bms = ms;
                    btx = tx;
                    bseg = sg;
                }
            }
            if (rs != RH_OK) break;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->timing = saved_timing;
        b->stage_tx = btx;
        b->stage_seg = bseg;
        rh_status up = upload_table(b);
        return rs != RH_OK ? rs : up;
    }
    int best_tx = b->tile_x, best_seg[3] = {0, b->seg[1], b->seg[2]};
    float best_ms = 1e30f;
    rh_status rs = RH_OK;
    for (int tx : {64, 32, 16}) {
        b->tile_x = tx;
        if ((rs = upload_table(b)) != RH_OK) break;
        float ms;
        if ((rs = time_class(0, &ms)) != RH_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best_tx = tx;
        }
    }
    b->tile_x = best_tx;
    for (int d = 1; d < 3 && rs == RH_OK; ++d) {
        best_ms = 1e30f;
        for (int sg : {16, 32, 48, 64, 128}) {
            b->seg[d] = sg;
            if ((rs = upload_table(b)) != RH_OK) break;
            float ms;
            if ((rs = time_class(d, &ms)) != RH_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_seg[d] = sg;
            }
        }
        b->seg[d] = best_seg[d];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->timing = saved_timing;
    rh_status up = upload_table(b);
    return rs != RH_OK ? rs : up;
}

rh_status rh_batch_set_timing(rh_batch* b, int enable) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (b->bound) (void)hipStreamSynchronize(b->stream);
    b->timing = enable != 0;
    b->timed.clear();
    b->event_next = 0;
    return RH_OK;
}

rh_status rh_batch_kernel_times(rh_batch* b, double* ms_out, long long* launches_out, int n) {
    if (!b) return fail(RH_E_INVAL, "batch is NULL");
    if (n < 0 || n > RH_KERNEL_CLASSES) return fail(RH_E_INVAL, "n out of range");
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    std::vector<double> ms(RH_KERNEL_CLASSES, 0.0);
    std::vector<long long> cnt(RH_KERNEL_CLASSES, 0);
    for (const TimedLaunch& t : b->timed) {
        float v = 0.f;
        if ((e = hipEventElapsedTime(&v, t.a, t.b)) != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
        ms[t.cls] += v;
        cnt[t.cls] += 1;
    }
    for (int i = 0; i < n; ++i) {
        if (ms_out) ms_out[i] = ms[i];
        if (launches_out) launches_out[i] = cnt[i];
    }
    return RH_OK;
}

}  // extern "C"

// ===========================================================================
// Adjoint of L and of one SSP-RK3 step
// ===========================================================================
namespace {

// out = (a1 X1 + a2 X2 + a3 X3) + s J(u)^T w (null X terms are skipped; they may
// alias out).  The recovery pack of u (six fields) goes to the bound workspace,
// from its own launch or from the whole-row x kernel; the x-axis kernel writes
// out from the linear combination and its own part, the y and z sweeps add
// theirs.
template <class T>
rh_status vjp_impl(rh_plan* p, double t, const T* u, const T* w, T* out, rh::Lin3<T> init, T s) {
    const long long N = 5 * p->ncell;
    const int n[3] = {p->d.nx, p->d.ny, p->d.nz};
    const double h[3] = {p->d.dx, p->d.dy, p->d.dz};
    T* pk = (T*)p->ws;
    rh::AdjArgs<T> base;
    std::memset(&base, 0, sizeof(base));
    base.u = u;
    base.w = w;
    base.ub = out;
    base.pk = pk;
    base.fstride = p->ncell;
    base.n[0] = n[0];
    base.n[1] = n[1];
    base.n[2] = n[2];
    base.eps = (T)(p->d.weno_eps > 0.0 ? p->d.weno_eps : 1e-6);
    base.scale = s;
    base.hb.t = t;
    base.hb.t0 = p->d.hubble_t0;
    base.hb.e0 = p->d.hubble_e0;
    base.hb.n0 = p->d.hubble_n0;
    base.hb.c0[0] = p->d.x0;
    base.hb.c0[1] = p->d.y0;
    base.hb.c0[2] = p->d.z0;
    base.hb.h[0] = h[0];
    base.hb.h[1] = h[1];
    base.hb.h[2] = h[2];
    // the whole-row x adjoint computes the pack of its cells and stores it
    const bool x_packs = n[0] > 1 && rh::adjoint_x_rows(n, p->d.bc[0]);
    rh_status st = RH_OK;
    if (!x_packs) {
        st = timed_launch(p, RH_KERNEL_OTHER,
                          [&] { return rh::launch_adjoint_pack<T>(u, pk, p->ncell, p->stream); }, "pack launch");
        if (st != RH_OK) return st;
    }
    if (n[0] > 1) {
        rh::AdjArgs<T> x = base;
        x.bc = p->d.bc[0];
        x.inv_h = (T)(1.0 / h[0]);
        st = timed_launch(p, RH_KERNEL_ADJOINT,
                          [&] { return rh::launch_adjoint_x<T>(p->d.scheme, x, init, p->stream); },
                          "adjoint sweep launch");
    } else if (init.X1 || init.X2 || init.X3) {
        st = timed_launch(p, RH_KERNEL_OTHER, [&] {
            return rh::launch_lincomb<T>(out, N, init.a1, init.X1, init.a2, init.X2, init.a3, init.X3, (T)0,
                                         nullptr, p->stream);
        }, "combine launch");
    } else {
        st = timed_launch(p, RH_KERNEL_OTHER, [&] { return rh::launch_fill_zero<T>(out, N, p->stream); },
                          "fill launch");
    }
    if (st != RH_OK) return st;
    for (int d = 1; d < 3; ++d) {
        if (n[d] < 2) continue;   // a one-cell axis contributes nothing to L
        rh::AdjArgs<T> q = base;
        q.bc = p->d.bc[d];
        q.inv_h = (T)(1.0 / h[d]);
        st = timed_launch(p, RH_KERNEL_ADJOINT,
                          [&] { return rh::launch_adjoint_sweep<T>(d, p->d.scheme, q, p->stream); },
                          "adjoint sweep launch");
        if (st != RH_OK) return st;
    }
    return RH_OK;
}

// Adjoint of one step given its stage states u1, u2 (b2, b1: scratch states)
template <class T>
rh_status step_vjp_core(rh_plan* p, double t, double dt, const T* un, const T* u1, const T* u2, const T* bin,
                        T* bout, T* b2, T* b1) {
    const T td = (T)dt;
    rh_status st;
    // b2 = 2/3 b + 2/3 dt J(u2)^T b
    const rh::Lin3<T> i2 = {(T)(2.0 / 3.0), (T)0, (T)0, bin, nullptr, nullptr};
    if ((st = vjp_impl<T>(p, t + 0.5 * dt, u2, bin, b2, i2, (T)(2.0 / 3.0) * td)) != RH_OK) return st;
    // b1 = 1/4 b2 + 1/4 dt J(u1)^T b2
    const rh::Lin3<T> i1 = {(T)0.25, (T)0, (T)0, b2, nullptr, nullptr};
    if ((st = vjp_impl<T>(p, t + dt, u1, b2, b1, i1, (T)0.25 * td)) != RH_OK) return st;
    // out = (1/3 b + 3/4 b2 + b1) + dt J(un)^T b1; the forward's last stage is
    // u^n + c (v - u^n) with c = 2/3 rounded, so its weight on u^n is 1 - c
    // (exact in both precisions) rather than 1/3 rounded
    const rh::Lin3<T> i0 = {(T)1 - (T)(2.0 / 3.0), (T)0.75, (T)1, bin, b2, b1};
    return vjp_impl<T>(p, t, un, b1, bout, i0, td);
}

// The stage states are recomputed into scratch[0..1]; b2 goes to scratch[2]
// and b1 reuses u2's slot once J(u2) has been applied.
template <class T>
rh_status step_vjp_impl(rh_plan* p, double t, double dt, const T* un, const T* bin, T* bout, T* scratch) {
    const size_t S = 5 * (size_t)p->ncell;
    T* u1 = scratch;
    T* u2 = scratch + S;
    T* Lc = (T*)p->ws + 2 * S;   // the bound workspace's L accumulator
    rh_status st = evaluate<T>(p, un, un, Lc, u1, t, dt, rh::STAGE_1);
    if (st == RH_OK) st = evaluate<T>(p, u1, un, Lc, u2, t + dt, dt, rh::STAGE_2);
    if (st != RH_OK) return st;
    return step_vjp_core<T>(p, t, dt, un, u1, u2, bin, bout, scratch + 2 * S, u2);
}

// [a, a + na) and [b, b + nb) intersect
bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* x = (const char*)a;
    const char* y = (const char*)b;
    return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

rh_status rh_apply_vjp(rh_plan* p, double t, const void* u, const void* w, void* out) {
    TraceRange trace("rh_apply_vjp");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!adjoint_supported(p->d))
        return fail(RH_E_NOTSUP, "the adjoint covers the WENO schemes with the conformal fluid and global splitting");
    if (!u || !w || !out) return fail(RH_E_INVAL, "NULL buffer");
    const size_t sb = rh_state_bytes(p);
    if (overlaps(out, sb, u, sb) || overlaps(out, sb, w, sb)) return fail(RH_E_INVAL, "out aliases u or w");
    if (overlaps(p->ws, 3 * sb, u, sb) || overlaps(p->ws, 3 * sb, w, sb) || overlaps(p->ws, 3 * sb, out, sb))
        return fail(RH_E_INVAL, "an operand aliases the bound workspace");
    if (is_fp32(p)) {
        const rh::Lin3<float> none = {0.0f, 0.0f, 0.0f, nullptr, nullptr, nullptr};
        return vjp_impl<float>(p, t, (const float*)u, (const float*)w, (float*)out, none, 1.0f);
    }
    const rh::Lin3<double> none = {0.0, 0.0, 0.0, nullptr, nullptr, nullptr};
    return vjp_impl<double>(p, t, (const double*)u, (const double*)w, (double*)out, none, 1.0);
}

rh_status rh_step_store(rh_plan* p, double dt, double* t_inout, void* stages) {
    TraceRange trace("rh_step_store");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!t_inout || !stages) return fail(RH_E_INVAL, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RH_E_INVAL, "dt must be > 0");
    const size_t sb = rh_state_bytes(p);
    if (overlaps(stages, 2 * sb, p->state, sb) || overlaps(stages, 2 * sb, p->ws, 3 * sb))
        return fail(RH_E_INVAL, "stages alias the bound state or workspace");
    st = is_fp32(p) ? step_impl<float>(p, dt, 1, *t_inout, (float*)stages)
                    : step_impl<double>(p, dt, 1, *t_inout, (double*)stages);
    if (st == RH_OK) *t_inout += dt;
    return st;
}

rh_status rh_step_store_n(rh_plan* p, double dt, int n_steps, double* t_inout, void* store) {
    TraceRange trace("rh_step_store_n");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!t_inout || (!store && n_steps != 0)) return fail(RH_E_INVAL, "NULL argument");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RH_E_INVAL, "dt must be > 0");
    if (n_steps < 0) return fail(RH_E_INVAL, "n_steps must be >= 0");
    const size_t sb = rh_state_bytes(p);
    if (n_steps > 0 && (size_t)n_steps > SIZE_MAX / (3 * sb)) return fail(RH_E_INVAL, "store size overflows");
    const size_t total = 3 * sb * (size_t)n_steps;
    if (n_steps > 0 && (overlaps(store, total, p->state, sb) || overlaps(store, total, p->ws, 3 * sb)))
        return fail(RH_E_INVAL, "store aliases the bound state or workspace");
    // step times as rh_step takes them (dt added once per step)
    double t = *t_inout;
    for (int k = 0; k < n_steps; ++k) {
        char* sk = (char*)store + 3 * sb * (size_t)k;
        const hipError_t e = hipMemcpyAsync(sk, p->state, sb, hipMemcpyDeviceToDevice, p->stream);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
        st = is_fp32(p) ? step_impl<float>(p, dt, 1, t, (float*)(sk + sb))
                        : step_impl<double>(p, dt, 1, t, (double*)(sk + sb));
        if (st != RH_OK) return st;
        t += dt;
    }
    *t_inout += n_steps * dt;
    return RH_OK;
}

rh_status rh_step_vjp_stored(rh_plan* p, double t, double dt, const void* u_n, const void* stages,
                             const void* ubar_in, void* ubar_out, void* scratch) {
    TraceRange trace("rh_step_vjp_stored");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!adjoint_supported(p->d))
        return fail(RH_E_NOTSUP, "the adjoint covers the WENO schemes with the conformal fluid and global splitting");
    if (!u_n || !stages || !ubar_in || !ubar_out || !scratch) return fail(RH_E_INVAL, "NULL buffer");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RH_E_INVAL, "dt must be > 0");
    const size_t sb = rh_state_bytes(p);
    if (overlaps(scratch, 2 * sb, u_n, sb) || overlaps(scratch, 2 * sb, stages, 2 * sb) ||
        overlaps(scratch, 2 * sb, ubar_in, sb) || overlaps(scratch, 2 * sb, ubar_out, sb))
        return fail(RH_E_INVAL, "scratch aliases an operand");
    if (overlaps(ubar_out, sb, u_n, sb) || overlaps(ubar_out, sb, stages, 2 * sb))
        return fail(RH_E_INVAL, "ubar_out aliases u_n or the stages");
    const char* ws = (const char*)p->ws;
    if (overlaps(ws, 3 * sb, u_n, sb) || overlaps(ws, 3 * sb, stages, 2 * sb) || overlaps(ws, 3 * sb, ubar_in, sb) ||
        overlaps(ws, 3 * sb, ubar_out, sb) || overlaps(ws, 3 * sb, scratch, 2 * sb))
        return fail(RH_E_INVAL, "an operand aliases the bound workspace");
    const size_t S = 5 * (size_t)p->ncell;
    if (is_fp32(p)) {
        const float* u1 = (const float*)stages;
        float* sc = (float*)scratch;
        return step_vjp_core<float>(p, t, dt, (const float*)u_n, u1, u1 + S, (const float*)ubar_in,
                                    (float*)ubar_out, sc, sc + S);
    }
    const double* u1 = (const double*)stages;
    double* sc = (double*)scratch;
    return step_vjp_core<double>(p, t, dt, (const double*)u_n, u1, u1 + S, (const double*)ubar_in,
                                 (double*)ubar_out, sc, sc + S);
}

size_t rh_vjp_workspace_bytes(const rh_plan* p) { return p ? 3 * rh_state_bytes(p) : 0; }

rh_status rh_step_vjp(rh_plan* p, double t, double dt, const void* u_n, const void* ubar_in,
                      void* ubar_out, void* scratch) {
    TraceRange trace("rh_step_vjp");
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!adjoint_supported(p->d))
        return fail(RH_E_NOTSUP, "the adjoint covers the WENO schemes with the conformal fluid and global splitting");
    if (!u_n || !ubar_in || !ubar_out || !scratch) return fail(RH_E_INVAL, "NULL buffer");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RH_E_INVAL, "dt must be > 0");
    const size_t sb = rh_state_bytes(p);
    if (overlaps(scratch, 3 * sb, u_n, sb) || overlaps(scratch, 3 * sb, ubar_in, sb) ||
        overlaps(scratch, 3 * sb, ubar_out, sb))
        return fail(RH_E_INVAL, "scratch aliases an operand");
    if (overlaps(ubar_out, sb, u_n, sb)) return fail(RH_E_INVAL, "ubar_out aliases u_n");
    const char* ws = (const char*)p->ws;
    if (overlaps(ws, 3 * sb, u_n, sb) || overlaps(ws, 3 * sb, ubar_in, sb) ||
        overlaps(ws, 3 * sb, ubar_out, sb) || overlaps(ws, 3 * sb, scratch, 3 * sb))
        return fail(RH_E_INVAL, "an operand aliases the bound workspace");
    return is_fp32(p) ? step_vjp_impl<float>(p, t, dt, (const float*)u_n, (const float*)ubar_in,
                                             (float*)ubar_out, (float*)scratch)
                      : step_vjp_impl<double>(p, t, dt, (const double*)u_n, (const double*)ubar_in,
                                              (double*)ubar_out, (double*)scratch);
}

}  // extern "C"

