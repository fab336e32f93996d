"""Python binding of the C ABI in include/rh.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: all work runs in the gfx950 kernels of librh.so.
PyTorch is used only to own device memory and to supply the HIP stream.

The binding fails loudly (ImportError) when librh.so has not been built; there
is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librh.so")

RH_OK, RH_E_INVAL, RH_E_NOMEM, RH_E_HIP, RH_E_STATE, RH_E_NOTSUP, RH_E_PHYS = 0, -1, -2, -3, -4, -5, -6
RH_PREC_FP64, RH_PREC_FP32 = 0, 1
RH_BC_PERIODIC, RH_BC_OUTFLOW, RH_BC_HUBBLE = 0, 1, 2
RH_FIELDS_CONSERVED, RH_FIELDS_PRIMITIVE = 0, 1
RH_KERNEL_SWEEP_X, RH_KERNEL_SWEEP_Y, RH_KERNEL_SWEEP_Z, RH_KERNEL_OTHER, RH_KERNEL_ADJOINT = 0, 1, 2, 3, 4
RH_KERNEL_SWEEP_XY = 5
RH_KERNEL_STAGE = 6
RH_KERNEL_CLASSES = 7
KERNEL_NAMES = ("sweep_x", "sweep_y", "sweep_z", "other", "adjoint", "sweep_xy", "stage")
RH_PATH_AUTO, RH_PATH_SWEEPS, RH_PATH_STAGE = 0, 1, 2
RH_SCHEME_MUSTA = 2
RH_LIMITER_MINMOD, RH_LIMITER_MC, RH_LIMITER_VANLEER, RH_LIMITER_SUPERBEE, RH_LIMITER_NONE = 0, 1, 2, 3, 4
RH_SPLIT_GLOBAL, RH_SPLIT_LOCAL = 0, 1
RH_EOS_CONFORMAL, RH_EOS_IDEAL = 0, 1
RH_NOALLOC_MAX_BYTES = 4294967295


class rh_grid_desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("scheme", ctypes.c_int), ("precision", ctypes.c_int), ("bc", ctypes.c_int * 3),
                ("weno_eps", ctypes.c_double), ("hubble_t0", ctypes.c_double),
                ("hubble_e0", ctypes.c_double), ("hubble_n0", ctypes.c_double),
                ("strict", ctypes.c_int), ("limiter", ctypes.c_int), ("musta_stages", ctypes.c_int),
                ("musta_cfl", ctypes.c_double), ("flux_split", ctypes.c_int), ("eos", ctypes.c_int),
                ("eos_gamma", ctypes.c_double)]


class RHError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("rh status %d: %s" % (status, message))
        self.status = status


_lib = None


def library():
    """Load librh.so (built by paper_1604_03360_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librh.so is not built (run python -m paper_1604_03360_amd.build); "
                              "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double
        pp = ctypes.POINTER(ctypes.c_void_p)
        L.rh_last_error.restype = ctypes.c_char_p
        L.rh_version.restype = ctypes.c_char_p
        L.rh_plan_create.argtypes = [pp, ctypes.POINTER(rh_grid_desc)]
        L.rh_plan_destroy.argtypes = [vp]
        L.rh_plan_destroy.restype = None
        L.rh_state_bytes.argtypes = [vp]
        L.rh_state_bytes.restype = ctypes.c_size_t
        L.rh_workspace_bytes.argtypes = [vp]
        L.rh_workspace_bytes.restype = ctypes.c_size_t
        L.rh_bind.argtypes = [vp, vp, vp, vp]
        L.rh_set_fields.argtypes = [vp, vp, i]
        L.rh_get_fields.argtypes = [vp, vp, i]
        L.rh_apply_L.argtypes = [vp, d, vp]
        L.rh_step.argtypes = [vp, d, i, dp]
        L.rh_totals.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong)]
        L.rh_totals_integrated.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong)]
        L.rh_reset_counters.argtypes = [vp]
        L.rh_set_timing.argtypes = [vp, i]
        L.rh_kernel_times.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_longlong), i]
        L.rh_apply_vjp.argtypes = [vp, d, vp, vp, vp]
        L.rh_vjp_workspace_bytes.argtypes = [vp]
        L.rh_vjp_workspace_bytes.restype = ctypes.c_size_t
        L.rh_step_vjp.argtypes = [vp, d, d, vp, vp, vp, vp]
        L.rh_step_store.argtypes = [vp, d, ctypes.POINTER(d), vp]
        L.rh_step_store_n.argtypes = [vp, d, i, ctypes.POINTER(d), vp]
        L.rh_set_graph.argtypes = [vp, i]
        L.rh_step_vjp_stored.argtypes = [vp, d, d, vp, vp, vp, vp, vp]
        llp = ctypes.POINTER(ctypes.c_longlong)
        ip = ctypes.POINTER(ctypes.c_int)
        L.rh_batch_create.argtypes = [pp, i, ctypes.POINTER(rh_grid_desc)]
        L.rh_batch_destroy.argtypes = [vp]
        L.rh_batch_destroy.restype = None
        L.rh_batch_offsets.argtypes = [vp, llp]
        L.rh_batch_state_bytes.argtypes = [vp]
        L.rh_batch_state_bytes.restype = ctypes.c_size_t
        L.rh_batch_workspace_bytes.argtypes = [vp]
        L.rh_batch_workspace_bytes.restype = ctypes.c_size_t
        L.rh_batch_bind.argtypes = [vp, vp, vp, vp]
        L.rh_batch_set_fields.argtypes = [vp, vp, i]
        L.rh_batch_get_fields.argtypes = [vp, vp, i]
        L.rh_batch_step.argtypes = [vp, d, i, dp]
        L.rh_batch_totals.argtypes = [vp, dp, llp]
        L.rh_batch_totals_integrated.argtypes = [vp, dp, llp]
        L.rh_batch_set_graph.argtypes = [vp, i]
        L.rh_batch_set_tuning.argtypes = [vp, i, i, i]
        L.rh_batch_get_tuning.argtypes = [vp, ip, ip, ip]
        L.rh_batch_autotune.argtypes = [vp, i]
        L.rh_batch_set_path.argtypes = [vp, i]
        L.rh_batch_get_path.argtypes = [vp, ip]
        L.rh_batch_set_stage_tuning.argtypes = [vp, i, i]
        L.rh_batch_get_stage_tuning.argtypes = [vp, ip, ip]
        L.rh_set_path.argtypes = [vp, i]
        L.rh_get_path.argtypes = [vp, ip]
        L.rh_set_stage_tuning.argtypes = [vp, i, i]
        L.rh_get_stage_tuning.argtypes = [vp, ip, ip]
        L.rh_totals_noalloc.argtypes = [vp, i, ctypes.c_longlong, vp, vp]
        L.rh_batch_set_timing.argtypes = [vp, i]
        L.rh_batch_kernel_times.argtypes = [vp, dp, llp, i]
        _lib = L
    return _lib


def _check(status):
    if status != RH_OK:
        raise RHError(status, library().rh_last_error().decode())
    return status


def rh_version():
    return library().rh_version().decode()


def rh_last_error():
    return library().rh_last_error().decode()


def rh_plan_create(desc):
    plan = ctypes.c_void_p()
    _check(library().rh_plan_create(ctypes.byref(plan), ctypes.byref(desc)))
    return plan


def rh_plan_destroy(plan):
    library().rh_plan_destroy(plan)


def rh_state_bytes(plan):
    return library().rh_state_bytes(plan)


def rh_workspace_bytes(plan):
    return library().rh_workspace_bytes(plan)


def rh_bind(plan, state_ptr, workspace_ptr, stream_ptr):
    _check(library().rh_bind(plan, ctypes.c_void_p(state_ptr), ctypes.c_void_p(workspace_ptr),
                             ctypes.c_void_p(stream_ptr)))


def rh_set_fields(plan, src_ptr, kind):
    _check(library().rh_set_fields(plan, ctypes.c_void_p(src_ptr), kind))


def rh_get_fields(plan, dst_ptr, kind):
    _check(library().rh_get_fields(plan, ctypes.c_void_p(dst_ptr), kind))


def rh_apply_L(plan, t, L_ptr):
    _check(library().rh_apply_L(plan, float(t), ctypes.c_void_p(L_ptr)))


def rh_step(plan, dt, n_steps, t):
    tt = ctypes.c_double(t)
    _check(library().rh_step(plan, float(dt), int(n_steps), ctypes.byref(tt)))
    return tt.value


def rh_totals(plan):
    out = (ctypes.c_double * 5)()
    cnt = (ctypes.c_longlong * 2)()
    _check(library().rh_totals(plan, out, cnt))
    return list(out), list(cnt)


def rh_totals_integrated(plan):
    out = (ctypes.c_double * 5)()
    cnt = (ctypes.c_longlong * 2)()
    _check(library().rh_totals_integrated(plan, out, cnt))
    return list(out), list(cnt)


def rh_totals_noalloc(state_ptr, precision, ncell, out_ptr, stream_ptr):
    """Enqueue the FP64 totals of a state [5][ncell] into the device buffer out_ptr[6]."""
    _check(library().rh_totals_noalloc(state_ptr, precision, ncell, out_ptr, stream_ptr))


def rh_reset_counters(plan):
    _check(library().rh_reset_counters(plan))


def rh_set_timing(plan, enable):
    _check(library().rh_set_timing(plan, int(bool(enable))))


def rh_kernel_times(plan):
    ms = (ctypes.c_double * RH_KERNEL_CLASSES)()
    cnt = (ctypes.c_longlong * RH_KERNEL_CLASSES)()
    _check(library().rh_kernel_times(plan, ms, cnt, RH_KERNEL_CLASSES))
    return {KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(RH_KERNEL_CLASSES)}


def rh_apply_vjp(plan, t, u_ptr, w_ptr, out_ptr):
    _check(library().rh_apply_vjp(plan, float(t), ctypes.c_void_p(u_ptr), ctypes.c_void_p(w_ptr),
                                  ctypes.c_void_p(out_ptr)))


def rh_vjp_workspace_bytes(plan):
    return library().rh_vjp_workspace_bytes(plan)


def rh_step_vjp(plan, t, dt, un_ptr, bin_ptr, bout_ptr, scratch_ptr):
    _check(library().rh_step_vjp(plan, float(t), float(dt), ctypes.c_void_p(un_ptr),
                                 ctypes.c_void_p(bin_ptr), ctypes.c_void_p(bout_ptr),
                                 ctypes.c_void_p(scratch_ptr)))


def rh_set_graph(plan, enable):
    _check(library().rh_set_graph(plan, 1 if enable else 0))


def rh_step_store(plan, dt, t, stages_ptr):
    tt = ctypes.c_double(t)
    _check(library().rh_step_store(plan, float(dt), ctypes.byref(tt), ctypes.c_void_p(stages_ptr)))
    return tt.value


def rh_step_store_n(plan, dt, n_steps, t, store_ptr):
    tt = ctypes.c_double(t)
    _check(library().rh_step_store_n(plan, float(dt), int(n_steps), ctypes.byref(tt),
                                     ctypes.c_void_p(store_ptr)))
    return tt.value


def rh_step_vjp_stored(plan, t, dt, un_ptr, stages_ptr, bin_ptr, bout_ptr, scratch_ptr):
    _check(library().rh_step_vjp_stored(plan, float(t), float(dt), ctypes.c_void_p(un_ptr),
                                        ctypes.c_void_p(stages_ptr), ctypes.c_void_p(bin_ptr),
                                        ctypes.c_void_p(bout_ptr), ctypes.c_void_p(scratch_ptr)))


def make_desc(shape, h, c0, scheme=5, precision=RH_PREC_FP64, bc=(RH_BC_PERIODIC,) * 3,
              eps=1e-6, hub=(10.0, 1.0, 0.5), strict=False, limiter=RH_LIMITER_MINMOD, musta_stages=0,
              musta_cfl=0.0, flux_split=RH_SPLIT_GLOBAL, eos=RH_EOS_CONFORMAL, eos_gamma=0.0):
    d = rh_grid_desc()
    d.limiter = int(limiter)
    d.musta_stages = int(musta_stages)
    d.musta_cfl = float(musta_cfl)
    d.flux_split = int(flux_split)
    d.eos = int(eos)
    d.eos_gamma = float(eos_gamma)
    d.nx, d.ny, d.nz = (int(s) for s in shape)
    d.dx, d.dy, d.dz = (float(v) for v in h)
    d.x0, d.y0, d.z0 = (float(v) for v in c0)
    d.scheme = int(scheme)
    d.precision = int(precision)
    for a in range(3):
        d.bc[a] = int(bc[a])
    d.weno_eps = float(eps)
    d.hubble_t0, d.hubble_e0, d.hubble_n0 = (float(v) for v in hub)
    d.strict = int(bool(strict))
    return d


def scheme_options(spec):
    """make_desc keywords of the scheme options a workload spec carries (MUSTA-FORCE
    limiter, stage count and local Courant number; local splitting; equation of state)."""
    out = {}
    if "limiter" in spec:
        out["limiter"] = spec["limiter"]
    if "musta_k" in spec:
        out["musta_stages"] = spec["musta_k"]
    if "musta_cfl" in spec:
        out["musta_cfl"] = spec["musta_cfl"]
    if spec.get("lf_local"):
        out["flux_split"] = RH_SPLIT_LOCAL
    if "eos" in spec:
        out["eos"] = spec["eos"]
    if "gamma" in spec:
        out["eos_gamma"] = spec["gamma"]
    return out


class Hydro:
    """One grid on the GPU: torch owns the state and workspace tensors, the
    library does all the work on torch's current stream."""

    def __init__(self, shape, h, c0, scheme=5, precision=RH_PREC_FP64, bc=(RH_BC_PERIODIC,) * 3,
                 eps=1e-6, hub=(10.0, 1.0, 0.5), strict=False, device="cuda", t=0.0, **scheme_opts):
        import torch
        self.torch = torch
        self.shape = tuple(int(s) for s in shape)
        self.desc = make_desc(shape, h, c0, scheme, precision, bc, eps, hub, strict, **scheme_opts)
        self.plan = rh_plan_create(self.desc)
        self.dtype = torch.float32 if precision == RH_PREC_FP32 else torch.float64
        nx, ny, nz = self.shape
        self.device = torch.device(device)
        self.state = torch.zeros((5, nz, ny, nx), dtype=self.dtype, device=self.device)
        self.workspace = torch.zeros((3, 5, nz, ny, nx), dtype=self.dtype, device=self.device)
        assert self.state.numel() * self.state.element_size() == rh_state_bytes(self.plan)
        assert self.workspace.numel() * self.workspace.element_size() == rh_workspace_bytes(self.plan)
        self.t = float(t)
        self.bind()

    @classmethod
    def from_spec(cls, spec, precision=RH_PREC_FP64, scheme=None, **kw):
        opts = scheme_options(spec)
        opts.update(kw)
        return cls(spec["shape"], spec["h"], spec["c0"], scheme=scheme or spec["order"],
                   precision=precision, bc=spec["bc"], eps=spec.get("eps", 1e-6),
                   hub=spec.get("hub", (10.0, 1.0, 0.5)), t=spec.get("t0", 0.0), **opts)

    def stream_ptr(self):
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def bind(self):
        rh_bind(self.plan, self.state.data_ptr(), self.workspace.data_ptr(), self.stream_ptr())

    def set_primitive(self, prim):
        src = self.torch.as_tensor(prim, dtype=self.torch.float64).to(self.device).contiguous()
        rh_set_fields(self.plan, src.data_ptr(), RH_FIELDS_PRIMITIVE)
        self.torch.cuda.current_stream(self.device).synchronize()

    def set_conserved(self, con):
        src = self.torch.as_tensor(con, dtype=self.torch.float64).to(self.device).contiguous()
        rh_set_fields(self.plan, src.data_ptr(), RH_FIELDS_CONSERVED)
        self.torch.cuda.current_stream(self.device).synchronize()

    def get(self, kind=RH_FIELDS_CONSERVED):
        nx, ny, nz = self.shape
        dst = self.torch.empty((5, nz, ny, nx), dtype=self.torch.float64, device=self.device)
        rh_get_fields(self.plan, dst.data_ptr(), kind)
        return dst.cpu().numpy()

    def apply_L(self, t=None):
        out = self.torch.empty_like(self.state)
        rh_apply_L(self.plan, self.t if t is None else t, out.data_ptr())
        return out

    def step(self, dt, n_steps=1):
        self.t = rh_step(self.plan, dt, n_steps, self.t)
        return self.t

    def totals(self, integrated=False):
        """FP64 sums of the conserved fields and the counters; with integrated,
        the sums times the cell volume."""
        return rh_totals_integrated(self.plan) if integrated else rh_totals(self.plan)

    def _dev(self, a):
        t = self.torch.as_tensor(a)
        return t.to(device=self.device, dtype=self.dtype).contiguous()

    def vjp(self, u, w, t=None):
        """J(u)^T w of L (device tensors or arrays of the plan layout)."""
        u, w = self._dev(u), self._dev(w)
        out = self.torch.empty_like(u)
        rh_apply_vjp(self.plan, self.t if t is None else t, u.data_ptr(), w.data_ptr(), out.data_ptr())
        return out

    def step_vjp(self, u_n, ubar, dt, t=None):
        """Adjoint of one SSP-RK3 step taken from u_n."""
        u_n, ubar = self._dev(u_n), self._dev(ubar)
        out = self.torch.empty_like(u_n)
        if getattr(self, "_vjp_scratch", None) is None:
            self._vjp_scratch = self.torch.empty((3,) + tuple(u_n.shape), dtype=self.dtype,
                                                 device=self.device)
        rh_step_vjp(self.plan, self.t if t is None else t, dt, u_n.data_ptr(), ubar.data_ptr(),
                    out.data_ptr(), self._vjp_scratch.data_ptr())
        return out

    def step_store(self, dt, stages=None):
        """One step that also returns its two stage states ([2][5][nz][ny][nx])."""
        if stages is None:
            stages = self.torch.empty((2,) + tuple(self.state.shape), dtype=self.dtype, device=self.device)
        self.t = rh_step_store(self.plan, dt, self.t, stages.data_ptr())
        return stages

    def step_store_n(self, dt, n_steps, store=None):
        """n_steps steps keeping (u_k, u1_k, u2_k) of each ([n][3][5][nz][ny][nx])."""
        if store is None:
            store = self.torch.empty((n_steps, 3) + tuple(self.state.shape), dtype=self.dtype,
                                     device=self.device)
        self.t = rh_step_store_n(self.plan, dt, n_steps, self.t, store.data_ptr())
        return store

    def step_vjp_stored(self, u_n, stages, ubar, dt, t=None):
        """Adjoint of one SSP-RK3 step from u_n whose stage states are given."""
        u_n, ubar = self._dev(u_n), self._dev(ubar)
        out = self.torch.empty_like(u_n)
        if getattr(self, "_vjp_scratch", None) is None:
            self._vjp_scratch = self.torch.empty((3,) + tuple(u_n.shape), dtype=self.dtype,
                                                 device=self.device)
        rh_step_vjp_stored(self.plan, self.t if t is None else t, dt, u_n.data_ptr(), stages.data_ptr(),
                           ubar.data_ptr(), out.data_ptr(), self._vjp_scratch.data_ptr())
        return out

    def close(self):
        if self.plan is not None:
            self.torch.cuda.current_stream(self.device).synchronize()
            rh_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Event-by-event batches
# ---------------------------------------------------------------------------
def rh_batch_create(descs):
    arr = (rh_grid_desc * len(descs))(*descs)
    b = ctypes.c_void_p()
    _check(library().rh_batch_create(ctypes.byref(b), len(descs), arr))
    return b


def rh_batch_destroy(batch):
    library().rh_batch_destroy(batch)


def rh_batch_offsets(batch, n_grids):
    out = (ctypes.c_longlong * (n_grids + 1))()
    _check(library().rh_batch_offsets(batch, out))
    return list(out)


def rh_batch_state_bytes(batch):
    return library().rh_batch_state_bytes(batch)


def rh_batch_workspace_bytes(batch):
    return library().rh_batch_workspace_bytes(batch)


def rh_batch_bind(batch, state_ptr, workspace_ptr, stream_ptr):
    _check(library().rh_batch_bind(batch, ctypes.c_void_p(state_ptr), ctypes.c_void_p(workspace_ptr),
                                   ctypes.c_void_p(stream_ptr)))


def rh_batch_set_fields(batch, src_ptr, kind):
    _check(library().rh_batch_set_fields(batch, ctypes.c_void_p(src_ptr), kind))


def rh_batch_get_fields(batch, dst_ptr, kind):
    _check(library().rh_batch_get_fields(batch, ctypes.c_void_p(dst_ptr), kind))


def rh_batch_step(batch, dt, n_steps, t):
    tt = ctypes.c_double(t)
    _check(library().rh_batch_step(batch, float(dt), int(n_steps), ctypes.byref(tt)))
    return tt.value


def rh_batch_totals(batch, n_grids):
    out = (ctypes.c_double * (5 * n_grids))()
    cnt = (ctypes.c_longlong * 2)()
    _check(library().rh_batch_totals(batch, out, cnt))
    return [list(out[5 * g:5 * g + 5]) for g in range(n_grids)], list(cnt)


def rh_batch_totals_integrated(batch, n_grids):
    out = (ctypes.c_double * (5 * n_grids))()
    cnt = (ctypes.c_longlong * 2)()
    _check(library().rh_batch_totals_integrated(batch, out, cnt))
    return [list(out[5 * g:5 * g + 5]) for g in range(n_grids)], list(cnt)


def rh_batch_set_graph(batch, enable):
    _check(library().rh_batch_set_graph(batch, int(bool(enable))))


def rh_batch_set_tuning(batch, tile_x, seg_y, seg_z):
    _check(library().rh_batch_set_tuning(batch, int(tile_x), int(seg_y), int(seg_z)))


def rh_batch_get_tuning(batch):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(library().rh_batch_get_tuning(batch, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def rh_batch_autotune(batch, reps=3):
    """Tune the launch shape of the batch's path; returns the stage tuning
    (tile_x, seg_z) on the fused-stage path, else the sweep tuning."""
    _check(library().rh_batch_autotune(batch, int(reps)))
    if rh_batch_get_path(batch) == RH_PATH_STAGE:
        return rh_batch_get_stage_tuning(batch)
    return rh_batch_get_tuning(batch)


def autotune_key(descs, path, device=""):
    """Text key of a tuned launch shape (independent of the order of the grids)."""
    sizes = {}
    for d in descs:
        k = "%dx%dx%d" % (d.nx, d.ny, d.nz)
        sizes[k] = sizes.get(k, 0) + 1
    d0 = descs[0]
    return "|".join([device, "path=%d" % path, "scheme=%d" % d0.scheme, "precision=%d" % d0.precision,
                     "eos=%d" % d0.eos, "split=%d" % d0.flux_split,
                     "sizes=" + ",".join("%s*%d" % (k, sizes[k]) for k in sorted(sizes))])


def load_autotune_cache(path):
    import json
    import os
    if not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            data = json.load(f)
    except ValueError:
        return {}
    return data if isinstance(data, dict) else {}


def store_autotune_cache(path, key, shape):
    import json
    import os
    data = load_autotune_cache(path)
    data[key] = list(shape)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def rh_batch_set_path(batch, path):
    _check(library().rh_batch_set_path(batch, int(path)))


def rh_batch_get_path(batch):
    a = ctypes.c_int()
    _check(library().rh_batch_get_path(batch, ctypes.byref(a)))
    return a.value


def rh_batch_set_stage_tuning(batch, tile_x, seg_z):
    _check(library().rh_batch_set_stage_tuning(batch, int(tile_x), int(seg_z)))


def rh_batch_get_stage_tuning(batch):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(library().rh_batch_get_stage_tuning(batch, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def rh_set_path(plan, path):
    _check(library().rh_set_path(plan, int(path)))


def rh_get_path(plan):
    a = ctypes.c_int()
    _check(library().rh_get_path(plan, ctypes.byref(a)))
    return a.value


def rh_set_stage_tuning(plan, tile_x, seg_z):
    _check(library().rh_set_stage_tuning(plan, int(tile_x), int(seg_z)))


def rh_get_stage_tuning(plan):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(library().rh_get_stage_tuning(plan, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def rh_batch_set_timing(batch, enable):
    _check(library().rh_batch_set_timing(batch, int(bool(enable))))


def rh_batch_kernel_times(batch):
    ms = (ctypes.c_double * RH_KERNEL_CLASSES)()
    cnt = (ctypes.c_longlong * RH_KERNEL_CLASSES)()
    _check(library().rh_batch_kernel_times(batch, ms, cnt, RH_KERNEL_CLASSES))
    return {KERNEL_NAMES[k]: (ms[k], cnt[k]) for k in range(RH_KERNEL_CLASSES)}


class Batch:
    """An event ensemble on the GPU: one concatenated state and workspace owned
    by torch; the library advances all grids with batched launches."""

    def __init__(self, specs, precision=RH_PREC_FP32, scheme=None, device="cuda"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.specs = specs
        self.descs = [make_desc(sp["shape"], sp["h"], sp["c0"], scheme or sp["order"], precision,
                                sp["bc"], sp.get("eps", 1e-6), sp.get("hub", (10.0, 1.0, 0.5)),
                                **scheme_options(sp))
                      for sp in specs]
        self.batch = rh_batch_create(self.descs)
        self.n = len(specs)
        self.offsets = rh_batch_offsets(self.batch, self.n)
        self.dtype = torch.float32 if precision == RH_PREC_FP32 else torch.float64
        total = self.offsets[-1]
        self.state = torch.zeros(total, dtype=self.dtype, device=self.device)
        self.workspace = torch.zeros(3 * total, dtype=self.dtype, device=self.device)
        self.t = float(specs[0].get("t0", 0.0))
        rh_batch_bind(self.batch, self.state.data_ptr(), self.workspace.data_ptr(),
                      torch.cuda.current_stream(self.device).cuda_stream)

    def _concat(self, arrays):
        import numpy as np
        buf = np.zeros(self.offsets[-1], dtype=np.float64)
        for g, a in enumerate(arrays):
            a = np.ascontiguousarray(a, dtype=np.float64).ravel()
            buf[self.offsets[g]:self.offsets[g] + a.size] = a
        return self.torch.from_numpy(buf).to(self.device)

    def set_primitive(self, prims):
        src = self._concat(prims)
        rh_batch_set_fields(self.batch, src.data_ptr(), RH_FIELDS_PRIMITIVE)
        self.torch.cuda.current_stream(self.device).synchronize()

    def get(self, kind=RH_FIELDS_CONSERVED):
        dst = self.torch.empty(self.offsets[-1], dtype=self.torch.float64, device=self.device)
        rh_batch_get_fields(self.batch, dst.data_ptr(), kind)
        host = dst.cpu().numpy()
        out = []
        for g, sp in enumerate(self.specs):
            nx, ny, nz = sp["shape"]
            out.append(host[self.offsets[g]:self.offsets[g] + 5 * nx * ny * nz].reshape(5, nz, ny, nx))
        return out

    def step(self, dt, n_steps=1):
        self.t = rh_batch_step(self.batch, dt, n_steps, self.t)
        return self.t

    def totals(self, integrated=False):
        if integrated:
            return rh_batch_totals_integrated(self.batch, self.n)
        return rh_batch_totals(self.batch, self.n)

    def tuning_key(self):
        """Key of this ensemble's launch-shape tuning: the evaluation path, scheme,
        precision, equation of state, splitting and the multiset of grid sizes."""
        return autotune_key(self.descs, rh_batch_get_path(self.batch), self.device_name())

    def device_name(self):
        return self.torch.cuda.get_device_name(self.device)

    def autotune(self, reps=2, cache=None):
        """Pick the launch shape of the batch's path: from the JSON file `cache`
        when it holds an entry for this ensemble's key, else by timing the
        candidates (rh_batch_autotune) and storing the result there.  Returns
        (shape, "cache" or "timed")."""
        key = self.tuning_key()
        path = rh_batch_get_path(self.batch)
        if cache is not None:
            entry = load_autotune_cache(cache).get(key)
            if entry is not None:
                if path == RH_PATH_STAGE:
                    rh_batch_set_stage_tuning(self.batch, *entry)
                else:
                    rh_batch_set_tuning(self.batch, *entry)
                return tuple(entry), "cache"
        shape = tuple(rh_batch_autotune(self.batch, reps))
        if cache is not None:
            store_autotune_cache(cache, key, shape)
        return shape, "timed"

    def close(self):
        if self.batch is not None:
            self.torch.cuda.current_stream(self.device).synchronize()
            rh_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
