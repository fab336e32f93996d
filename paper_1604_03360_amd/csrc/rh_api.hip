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
#include <string>
#include <vector>

#include "../../include/rh.h"
#include "rh_internal.hpp"

namespace {

thread_local std::string g_last_error;

rh_status fail(rh_status code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

rh_status hip_fail(hipError_t e, const char* what) {
    return fail(RH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
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
        if (stage == rh::STAGE_WRITE_L) {
            hipError_t e = hipMemsetAsync(lacc, 0, 5 * p->ncell * sizeof(T), p->stream);
            return e == hipSuccess ? RH_OK : hip_fail(e, "hipMemsetAsync");
        }
        return timed_launch(p, RH_KERNEL_OTHER, [&] { return rh::launch_combine<T>(a, p->stream); },
                            "combine launch");
    }
    for (int i = 0; i < na; ++i) {
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
rh_status step_impl(rh_plan* p, double dt, int nsteps, double t) {
    const size_t S = 5 * (size_t)p->ncell;
    T* U0 = (T*)p->state;
    T* U1 = (T*)p->ws;
    T* U2 = U1 + S;
    T* Lc = U2 + S;
    for (int s = 0; s < nsteps; ++s) {
        rh_status st;
        st = evaluate<T>(p, U0, U0, Lc, U1, t, dt, rh::STAGE_1);
        if (st != RH_OK) return st;
        st = evaluate<T>(p, U1, U0, Lc, U2, t + dt, dt, rh::STAGE_2);
        if (st != RH_OK) return st;
        st = evaluate<T>(p, U2, U0, Lc, U0, t + 0.5 * dt, dt, rh::STAGE_3);
        if (st != RH_OK) return st;
        t += dt;
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
    if (d->scheme != 5 && d->scheme != 7) return fail(RH_E_INVAL, "scheme must be 5 or 7");
    if (d->precision != RH_PREC_FP64 && d->precision != RH_PREC_FP32)
        return fail(RH_E_INVAL, "unknown precision");
    if (d->weno_eps < 0.0) return fail(RH_E_INVAL, "weno_eps must be >= 0");
    const long long ny_nz = (long long)n[1] * n[2];
    if ((ny_nz + 3) / 4 > 65535LL * 64 && n[0] > 1) return fail(RH_E_INVAL, "grid too large");
    if ((long long)(n[1] + 3) / 4 > 65535 || (long long)(n[2] + 3) / 4 > 65535)
        return fail(RH_E_INVAL, "transverse axis too long for the launch grid");
    for (int a = 0; a < 3; ++a) {
        if (d->bc[a] == RH_BC_HUBBLE && !(d->hubble_t0 > 0.0))
            return fail(RH_E_INVAL, "HUBBLE boundaries need hubble_t0 > 0");
    }
    rh_plan* p = new (std::nothrow) rh_plan();
    if (!p) return fail(RH_E_NOMEM, "host allocation failed");
    p->d = *d;
    p->ghosts = (d->scheme + 1) / 2;
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
        return is_fp32(p) ? rh::launch_set_fields<float>((float*)p->state, src, kind, p->ncell, p->stream)
                          : rh::launch_set_fields<double>((double*)p->state, src, kind, p->ncell, p->stream);
    }, "set_fields launch");
}

rh_status rh_get_fields(rh_plan* p, double* dst, int kind) {
    rh_status st = check_bound(p);
    if (st != RH_OK) return st;
    if (!dst) return fail(RH_E_INVAL, "dst is NULL");
    if (kind != RH_FIELDS_CONSERVED && kind != RH_FIELDS_PRIMITIVE) return fail(RH_E_INVAL, "bad kind");
    return timed_launch(p, RH_KERNEL_OTHER, [&] {
        return is_fp32(p) ? rh::launch_get_fields<float>((const float*)p->state, dst, kind, p->ncell,
                                                         p->d_clamps, p->stream)
                          : rh::launch_get_fields<double>((const double*)p->state, dst, kind, p->ncell,
                                                          p->d_clamps, p->stream);
    }, "get_fields launch");
}

rh_status rh_apply_L(rh_plan* p, double t, void* L_out) {
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

rh_status rh_totals(rh_plan* p, double out[5], long long counters[2]) {
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
