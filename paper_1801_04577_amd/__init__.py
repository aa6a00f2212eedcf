"""Python binding of libclbm.so, the gfx950 library for the thermal cascaded LBM of
Fei & Luo (arXiv:1801.04577).

Argument marshalling only: every step of the method runs in the HIP kernels of
``csrc/`` behind the C ABI declared in ``include/clbm.h``. PyTorch supplies
device memory (the workspace and field tensors) and the HIP stream. The
functions below carry the C names; ``Solver`` and ``Batch`` are small
conveniences over them.

There is no fallback: if ``libclbm.so`` has not been built, loading fails.
"""
import ctypes
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libclbm.so")

CLBM_OK = 0
CLBM_ERR_NAN = -5
CLBM_FP32 = 0
CLBM_FP16_SHIFTED = 1
_KIND = {"periodic": 0, "wall": 1}
INST_STATUS = {0: "running", 1: "converged", 2: "diverged", 3: "max_steps"}


class ClbmError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__("%s failed: %s (status %d)" % (what, status_string(status), status))


class clbm_side(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("u_wall", ctypes.c_double), ("b1", ctypes.c_double),
                ("b2", ctypes.c_double), ("b3", ctypes.c_double)]


class clbm_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("precision", ctypes.c_int),
        ("nu", ctypes.c_double), ("alpha", ctypes.c_double),
        ("s_b", ctypes.c_double), ("s_4", ctypes.c_double), ("s_3", ctypes.c_double),
        ("lambda_0", ctypes.c_double), ("lambda_2", ctypes.c_double),
        ("g_beta", ctypes.c_double), ("T0", ctypes.c_double),
        ("Fx", ctypes.c_double), ("Fy", ctypes.c_double), ("Q", ctypes.c_double),
        ("viscous_heating", ctypes.c_int),
        ("side", clbm_side * 4),
    ]


class clbm_launch(ctypes.Structure):
    _fields_ = [("block_x", ctypes.c_int), ("block_y", ctypes.c_int),
                ("rows_per_thread", ctypes.c_int), ("xcd_remap", ctypes.c_int),
                ("steps_per_launch", ctypes.c_int), ("two_step_rows", ctypes.c_int)]


class clbm_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_long), ("K", ctypes.c_int), ("mass", ctypes.c_double),
        ("sum_u2", ctypes.c_double), ("sum_du2", ctypes.c_double), ("sum_T2", ctypes.c_double),
        ("sum_dT2", ctypes.c_double), ("res_u", ctypes.c_double), ("res_T", ctypes.c_double),
        ("dTdn", ctypes.c_double * 4), ("T_wall", ctypes.c_double * 4),
        ("wall_flux", ctypes.c_double * 4), ("nan_count", ctypes.c_long),
    ]

    def as_dict(self):
        return {"step": self.step, "K": self.K, "mass": self.mass, "sum_u2": self.sum_u2,
                "sum_du2": self.sum_du2, "sum_T2": self.sum_T2, "sum_dT2": self.sum_dT2,
                "res_u": self.res_u, "res_T": self.res_T, "dTdn": list(self.dTdn),
                "T_wall": list(self.T_wall), "wall_flux": list(self.wall_flux),
                "nan_count": self.nan_count}


class clbm_net_desc(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int), ("height", ctypes.c_int), ("width", ctypes.c_int),
                ("cin", ctypes.c_int), ("cout", ctypes.c_int), ("widths", ctypes.c_int * 4)]


class clbm_problem_code(ctypes.Structure):
    _fields_ = [("log10_ra", ctypes.c_float), ("pr", ctypes.c_float), ("q_star", ctypes.c_float),
                ("log2_aspect", ctypes.c_float), ("theta_wall", ctypes.c_float * 4),
                ("kind", ctypes.c_int * 4), ("u_scale", ctypes.c_float), ("t_scale", ctypes.c_float)]


class clbm_batch_launch(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int), ("tile_y", ctypes.c_int), ("persistent_wgs", ctypes.c_int),
                ("steps_per_launch", ctypes.c_int), ("xcd_bands", ctypes.c_int)]


_lib = None
_VP = ctypes.c_void_p
_FP = ctypes.c_void_p  # device float* passed as integer addresses


def _declare(L):
    P = ctypes.POINTER(clbm_params)
    st = ctypes.c_int
    sig = {
        "clbm_abi_version": (ctypes.c_int, []),
        "clbm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "clbm_derive_rates": (st, [P, ctypes.POINTER(ctypes.c_double)]),
        "clbm_workspace_bytes": (st, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "clbm_create": (st, [P, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
        "clbm_destroy": (None, [_VP]),
        "clbm_init_from_fields": (st, [_VP, _FP, _FP, _FP, _FP]),
        "clbm_step": (st, [_VP, ctypes.c_int]),
        "clbm_macros": (st, [_VP, _FP, _FP, _FP, _FP]),
        "clbm_populations": (st, [_VP, _FP, _FP]),
        "clbm_diagnostics": (st, [_VP, ctypes.POINTER(clbm_diag)]),
        "clbm_diagnostics_noalloc": (st, [_VP, ctypes.POINTER(clbm_diag)]),
        "clbm_state_bytes": (st, [_VP, ctypes.POINTER(ctypes.c_size_t)]),
        "clbm_save": (st, [_VP, _VP]),
        "clbm_load": (st, [_VP, _VP, ctypes.c_long]),
        "clbm_get_step": (st, [_VP, ctypes.POINTER(ctypes.c_long)]),
        "clbm_set_launch": (st, [_VP, ctypes.POINTER(clbm_launch)]),
        "clbm_get_launch": (st, [_VP, ctypes.POINTER(clbm_launch)]),
        "clbm_set_graph": (st, [_VP, ctypes.c_int]),
        "clbm_set_source_field": (st, [_VP, _VP]),
        "clbm_batch_set_source_field": (st, [_VP, ctypes.c_int, _VP]),
        "clbm_stream_copy": (st, [_VP, _VP, ctypes.c_size_t, _VP]),
        "clbm_net_param_count": (st, [ctypes.POINTER(clbm_net_desc), ctypes.POINTER(ctypes.c_size_t)]),
        "clbm_net_workspace_bytes": (st, [ctypes.POINTER(clbm_net_desc), ctypes.POINTER(ctypes.c_size_t)]),
        "clbm_net_create": (st, [ctypes.POINTER(clbm_net_desc), _VP, ctypes.c_size_t, _VP,
                                 ctypes.POINTER(_VP)]),
        "clbm_net_destroy": (None, [_VP]),
        "clbm_net_set_params": (st, [_VP, _VP]),
        "clbm_net_get_params": (st, [_VP, _VP]),
        "clbm_net_get_grads": (st, [_VP, _VP]),
        "clbm_net_forward": (st, [_VP, _VP, _VP]),
        "clbm_net_backward": (st, [_VP, _VP, ctypes.POINTER(ctypes.c_double)]),
        "clbm_net_adam": (st, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                               ctypes.c_int]),
        "clbm_resample_bilinear": (st, [_VP, ctypes.c_int, ctypes.c_int, _VP, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float), _VP]),
        "clbm_problem_encode": (st, [ctypes.POINTER(clbm_params), ctypes.POINTER(clbm_problem_code)]),
        "clbm_net_features": (st, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP]),
        "clbm_batch_workspace_bytes": (st, [ctypes.c_int, P, ctypes.POINTER(ctypes.c_size_t)]),
        "clbm_batch_create": (st, [ctypes.c_int, P, _VP, ctypes.c_size_t, _VP,
                                   ctypes.POINTER(clbm_batch_launch), ctypes.POINTER(_VP)]),
        "clbm_batch_destroy": (None, [_VP]),
        "clbm_batch_init": (st, [_VP, ctypes.c_int, _FP, _FP, _FP, _FP]),
        "clbm_batch_step": (st, [_VP, ctypes.c_int]),
        "clbm_batch_reset": (st, [_VP]),
        "clbm_batch_run": (st, [_VP, ctypes.c_long, ctypes.c_double, ctypes.c_int, ctypes.c_long,
                                ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_int)]),
        "clbm_batch_macros": (st, [_VP, ctypes.c_int, _FP, _FP, _FP, _FP]),
        "clbm_batch_residual": (st, [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]),
        "clbm_batch_diagnostics": (st, [_VP, ctypes.c_int, ctypes.POINTER(clbm_diag)]),
        "clbm_batch_autotune": (st, [_VP, ctypes.c_int, ctypes.c_char_p,
                                     ctypes.POINTER(clbm_batch_launch)]),
        "clbm_batch_tune_lookup": (st, [_VP, ctypes.c_char_p, ctypes.POINTER(clbm_batch_launch),
                                        ctypes.POINTER(ctypes.c_int)]),
        "clbm_batch_set_launch": (st, [_VP, ctypes.POINTER(clbm_batch_launch)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    return L


def lib():
    """Load libclbm.so. Raises if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError("libclbm.so is not built; run paper_1801_04577_amd/build.py "
                              "(or __graft_entry__.build())")
        _lib = _declare(ctypes.CDLL(LIBPATH))
    return _lib


def ensure_built():
    """Build the library only if it is missing, then load it."""
    if not os.path.exists(LIBPATH):
        from . import build as _build
        _build.build()
    return lib()


def status_string(status):
    try:
        return lib().clbm_status_string(int(status)).decode()
    except Exception:
        return "status %d" % status


def _check(status, what):
    if status != CLBM_OK:
        raise ClbmError(status, what)


def _nan_if_none(v):
    return float("nan") if v is None else float(v)


def make_params(prob, precision=CLBM_FP32):
    """clbm_params from a problem dict (see workloads/) -- marshalling only."""
    p = clbm_params()
    p.nx, p.ny = int(prob["nx"]), int(prob["ny"])
    p.precision = int(precision)
    p.nu, p.alpha = float(prob["nu"]), float(prob["alpha"])
    for k in ("s_b", "s_4", "s_3", "lambda_0", "lambda_2"):
        setattr(p, k, _nan_if_none(prob.get(k)))
    for k in ("g_beta", "T0", "Fx", "Fy", "Q"):
        setattr(p, k, float(prob.get(k, 0.0)))
    p.viscous_heating = int(bool(prob.get("viscous_heating", False)))
    for s, side in enumerate(prob["sides"]):
        p.side[s].kind = _KIND[side["kind"]]
        p.side[s].u_wall = float(side.get("u_wall", 0.0))
        p.side[s].b1 = float(side.get("b1", 0.0))
        p.side[s].b2 = float(side.get("b2", 1.0))
        p.side[s].b3 = float(side.get("b3", 0.0))
    return p


def _addr(t):
    return None if t is None else ctypes.c_void_p(int(t.data_ptr()))


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


# ---------------------------------------------------------------------------
# C-named wrappers
# ---------------------------------------------------------------------------

def clbm_abi_version():
    return lib().clbm_abi_version()


def clbm_derive_rates(params):
    out = (ctypes.c_double * 7)()
    _check(lib().clbm_derive_rates(ctypes.byref(params), out), "clbm_derive_rates")
    return list(out)


def clbm_workspace_bytes(params):
    n = ctypes.c_size_t()
    _check(lib().clbm_workspace_bytes(ctypes.byref(params), ctypes.byref(n)), "clbm_workspace_bytes")
    return n.value


def clbm_batch_workspace_bytes(params_list):
    arr = (clbm_params * len(params_list))(*params_list)
    n = ctypes.c_size_t()
    _check(lib().clbm_batch_workspace_bytes(len(params_list), arr, ctypes.byref(n)),
           "clbm_batch_workspace_bytes")
    return n.value


def clbm_stream_copy(dst, src, stream=None):
    """Device copy of src into dst (uint8/float tensors of equal byte size) by the
    library's streaming-copy kernel (bandwidth reference)."""
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    _check(lib().clbm_stream_copy(_addr(dst), _addr(src), nbytes, _stream_ptr(stream)),
           "clbm_stream_copy")


def _workspace(nbytes, device):
    import torch
    # 256-byte aligned by the caching allocator; keep the tensor alive with the handle.
    return torch.empty(int(nbytes), dtype=torch.uint8, device=device)


class Solver:
    """One lattice on the GPU. Fields are torch float32 tensors [ny][nx] on the device."""

    def __init__(self, prob, precision=CLBM_FP32, device="cuda", stream=None):
        import torch
        self.prob = prob
        self.nx, self.ny = int(prob["nx"]), int(prob["ny"])
        self.device = torch.device(device)
        self.params = make_params(prob, precision)
        self.precision = precision
        L = lib()
        self.workspace = _workspace(clbm_workspace_bytes(self.params), self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(L.clbm_create(ctypes.byref(self.params), _addr(self.workspace),
                             self.workspace.numel(), _stream_ptr(self.stream), ctypes.byref(h)),
               "clbm_create")
        self._h = h
        self._qfield = None
        if prob.get("Q_field") is not None:
            self.set_source_field(prob["Q_field"])

    def set_source_field(self, q):
        """Heat source per node added to Q (array-like [ny][nx], or None to remove it)."""
        t = None if q is None else self._f(q)
        self._qfield = t  # the kernels read it on every step
        _check(lib().clbm_set_source_field(self._h, _addr(t)), "clbm_set_source_field")

    def _f(self, a):
        import torch
        if a is None:
            return None
        t = torch.as_tensor(a, dtype=torch.float32, device=self.device)
        t = t.expand(self.ny, self.nx).contiguous() if t.dim() < 2 else t.contiguous()
        assert tuple(t.shape) == (self.ny, self.nx), t.shape
        return t

    def init(self, rho=None, ux=None, uy=None, T=None):
        fs = [self._f(a) for a in (rho, ux, uy, T)]
        _check(lib().clbm_init_from_fields(self._h, *[_addr(t) for t in fs]), "clbm_init_from_fields")
        self._keep = fs  # the kernel reads them asynchronously

    def step(self, n=1):
        _check(lib().clbm_step(self._h, int(n)), "clbm_step")

    @property
    def t(self):
        v = ctypes.c_long()
        _check(lib().clbm_get_step(self._h, ctypes.byref(v)), "clbm_get_step")
        return v.value

    def macros(self):
        import torch
        out = [torch.empty(self.ny, self.nx, dtype=torch.float32, device=self.device) for _ in range(4)]
        _check(lib().clbm_macros(self._h, *[_addr(t) for t in out]), "clbm_macros")
        return tuple(out)

    def populations(self):
        """Post-collision deviations (f* - w [9][ny][nx], g* - T0/5 [5][ny][nx])."""
        import torch
        f = torch.empty(9, self.ny, self.nx, dtype=torch.float32, device=self.device)
        g = torch.empty(5, self.ny, self.nx, dtype=torch.float32, device=self.device)
        _check(lib().clbm_populations(self._h, _addr(f), _addr(g)), "clbm_populations")
        return f, g

    def diagnostics(self, raise_on_nan=False, noalloc=False):
        """clbm_diagnostics, or with noalloc clbm_diagnostics_noalloc (partial sums in the
        library's own device array instead of the workspace)."""
        d = clbm_diag()
        name = "clbm_diagnostics_noalloc" if noalloc else "clbm_diagnostics"
        st = getattr(lib(), name)(self._h, ctypes.byref(d))
        if st == CLBM_ERR_NAN and not raise_on_nan:
            return d
        _check(st, name)
        return d

    def state_bytes(self):
        n = ctypes.c_size_t()
        _check(lib().clbm_state_bytes(self._h, ctypes.byref(n)), "clbm_state_bytes")
        return n.value

    def save(self):
        import torch
        buf = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        _check(lib().clbm_save(self._h, _addr(buf)), "clbm_save")
        return buf, self.t

    def load(self, buf, step):
        _check(lib().clbm_load(self._h, _addr(buf), int(step)), "clbm_load")

    def set_launch(self, block_x=256, block_y=1, rows_per_thread=1, xcd_remap=0, steps_per_launch=1,
                   two_step_rows=0):
        L = clbm_launch(int(block_x), int(block_y), int(rows_per_thread), int(xcd_remap),
                        int(steps_per_launch), int(two_step_rows))
        _check(lib().clbm_set_launch(self._h, ctypes.byref(L)), "clbm_set_launch")

    def get_launch(self):
        L = clbm_launch()
        _check(lib().clbm_get_launch(self._h, ctypes.byref(L)), "clbm_get_launch")
        return {"block_x": L.block_x, "block_y": L.block_y, "rows_per_thread": L.rows_per_thread,
                "xcd_remap": L.xcd_remap, "steps_per_launch": L.steps_per_launch,
                "two_step_rows": L.two_step_rows}

    def set_graph(self, steps_per_graph):
        _check(lib().clbm_set_graph(self._h, int(steps_per_graph)), "clbm_set_graph")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().clbm_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _launch_dict(L):
    return {"tile_x": L.tile_x, "tile_y": L.tile_y, "persistent_wgs": L.persistent_wgs,
            "steps_per_launch": L.steps_per_launch, "xcd_bands": L.xcd_bands}


class Batch:
    """Many lattices (own sizes and parameters) advanced together on the GPU."""

    def __init__(self, probs, device="cuda", stream=None, launch=None, precision=CLBM_FP32,
                 tune_cache=None):
        """precision: the storage type of every instance. launch: a dict of
        clbm_batch_launch fields; tune_cache: a cache file written by autotune, whose
        entry for this workload (if any) replaces the default launch."""
        import torch
        self.probs = list(probs)
        self.n = len(self.probs)
        self.device = torch.device(device)
        self.precision = precision
        self.params = (clbm_params * self.n)(*[make_params(p, precision) for p in self.probs])
        nbytes = ctypes.c_size_t()
        _check(lib().clbm_batch_workspace_bytes(self.n, self.params, ctypes.byref(nbytes)),
               "clbm_batch_workspace_bytes")
        self.workspace = _workspace(nbytes.value, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = None
        if launch:
            L = clbm_batch_launch(int(launch["tile_x"]), int(launch["tile_y"]),
                                  int(launch.get("persistent_wgs", 0)),
                                  int(launch.get("steps_per_launch", 1)),
                                  int(launch.get("xcd_bands", 1)))
        h = ctypes.c_void_p()
        _check(lib().clbm_batch_create(self.n, self.params, _addr(self.workspace),
                                       self.workspace.numel(), _stream_ptr(self.stream),
                                       ctypes.byref(L) if L is not None else None, ctypes.byref(h)),
               "clbm_batch_create")
        self._h = h
        self._keep = {}
        self._qfields = {}
        for i, p in enumerate(self.probs):
            if p.get("Q_field") is not None:
                self.set_source_field(i, p["Q_field"])
        self.tuned_from_cache = False
        if tune_cache and launch is None:
            cached = self.cached_launch(tune_cache)
            if cached is not None:
                self.set_launch(**cached)
                self.tuned_from_cache = True

    def cached_launch(self, cache_path):
        """The launch autotune stored for this workload in cache_path, or None."""
        L = clbm_batch_launch()
        found = ctypes.c_int()
        _check(lib().clbm_batch_tune_lookup(self._h, cache_path.encode(), ctypes.byref(L),
                                            ctypes.byref(found)), "clbm_batch_tune_lookup")
        return _launch_dict(L) if found.value else None

    def init(self, i, rho=None, ux=None, uy=None, T=None):
        import torch
        nx, ny = int(self.probs[i]["nx"]), int(self.probs[i]["ny"])
        fs = []
        for a in (rho, ux, uy, T):
            if a is None:
                fs.append(None)
                continue
            t = torch.as_tensor(a, dtype=torch.float32, device=self.device)
            t = t.expand(ny, nx).contiguous() if t.dim() < 2 else t.contiguous()
            assert tuple(t.shape) == (ny, nx), t.shape
            fs.append(t)
        _check(lib().clbm_batch_init(self._h, int(i), *[_addr(t) for t in fs]), "clbm_batch_init")
        self._keep[i] = fs

    def set_source_field(self, i, q):
        """Heat source per node of instance i added to its Q ([ny][nx], or None)."""
        import torch
        t = None
        if q is not None:
            nx, ny = int(self.probs[i]["nx"]), int(self.probs[i]["ny"])
            t = torch.as_tensor(q, dtype=torch.float32, device=self.device)
            t = t.expand(ny, nx).contiguous() if t.dim() < 2 else t.contiguous()
            assert tuple(t.shape) == (ny, nx), t.shape
        self._qfields[i] = t  # the kernels read it on every step
        _check(lib().clbm_batch_set_source_field(self._h, int(i), _addr(t)), "clbm_batch_set_source_field")

    def step(self, n=1):
        _check(lib().clbm_batch_step(self._h, int(n)), "clbm_batch_step")

    def run(self, max_steps, tol, K=1000, chunk=0, progress=None, reset=True, max_calls=0):
        """Runs every instance to tol (see clbm_batch_run), after clbm_batch_reset unless
        reset is False (then the previous run resumes). With chunk > 0 the run proceeds
        in calls of at most chunk steps and progress(steps, status) is called after each;
        max_calls > 0 stops after that many calls. Returns (steps, status) per instance;
        status names from INST_STATUS. With FP16 storage the residual floor is about 1e-6:
        choose tol above it."""
        if reset:
            _check(lib().clbm_batch_reset(self._h), "clbm_batch_reset")
        steps = (ctypes.c_long * self.n)()
        status = (ctypes.c_int * self.n)()
        calls = 0
        while True:
            _check(lib().clbm_batch_run(self._h, int(max_steps), float(tol), int(K), int(chunk), steps,
                                        status), "clbm_batch_run")
            calls += 1
            names = [INST_STATUS[s] for s in status]
            if progress is not None:
                progress(list(steps), names)
            if chunk <= 0 or "running" not in names or (max_calls and calls >= max_calls):
                return list(steps), names

    def macros(self, i):
        import torch
        nx, ny = int(self.probs[i]["nx"]), int(self.probs[i]["ny"])
        out = [torch.empty(ny, nx, dtype=torch.float32, device=self.device) for _ in range(4)]
        _check(lib().clbm_batch_macros(self._h, int(i), *[_addr(t) for t in out]), "clbm_batch_macros")
        return tuple(out)

    def diagnostics(self, i):
        d = clbm_diag()
        st = lib().clbm_batch_diagnostics(self._h, int(i), ctypes.byref(d))
        if st not in (CLBM_OK, CLBM_ERR_NAN):
            _check(st, "clbm_batch_diagnostics")
        return d

    def residual(self, i):
        out = (ctypes.c_double * 2)()
        _check(lib().clbm_batch_residual(self._h, int(i), out), "clbm_batch_residual")
        return out[0], out[1]

    def set_launch(self, tile_x, tile_y, persistent_wgs=0, steps_per_launch=1, xcd_bands=1):
        L = clbm_batch_launch(int(tile_x), int(tile_y), int(persistent_wgs), int(steps_per_launch),
                              int(xcd_bands))
        _check(lib().clbm_batch_set_launch(self._h, ctypes.byref(L)), "clbm_batch_set_launch")

    def autotune(self, steps=20, cache_path=None):
        best = clbm_batch_launch()
        path = cache_path.encode() if cache_path else None
        _check(lib().clbm_batch_autotune(self._h, int(steps), path, ctypes.byref(best)),
               "clbm_batch_autotune")
        return _launch_dict(best)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().clbm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Net:
    """The warm-start encoder-decoder on the GPU (BF16 MFMA kernels, FP32 master weights).
    Parameters are a flat float32 tensor in the canonical order of include/clbm.h."""

    def __init__(self, batch, height, width, cin, cout, widths, device="cuda", stream=None):
        import torch
        self.device = torch.device(device)
        self.desc = clbm_net_desc(int(batch), int(height), int(width), int(cin), int(cout),
                                  (ctypes.c_int * 4)(*[int(w) for w in widths]))
        self.shape_in = (int(batch), int(cin), int(height), int(width))
        self.shape_out = (int(batch), int(cout), int(height), int(width))
        n = ctypes.c_size_t()
        _check(lib().clbm_net_param_count(ctypes.byref(self.desc), ctypes.byref(n)), "clbm_net_param_count")
        self.nparams = n.value
        _check(lib().clbm_net_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(n)),
               "clbm_net_workspace_bytes")
        self.workspace = _workspace(n.value, self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(lib().clbm_net_create(ctypes.byref(self.desc), _addr(self.workspace), self.workspace.numel(),
                                     _stream_ptr(self.stream), ctypes.byref(h)), "clbm_net_create")
        self._h = h

    def set_params(self, params):
        import torch
        t = torch.as_tensor(params, dtype=torch.float32, device=self.device).contiguous()
        assert t.numel() == self.nparams
        _check(lib().clbm_net_set_params(self._h, _addr(t)), "clbm_net_set_params")
        self._keep_params = t

    def params(self):
        import torch
        t = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check(lib().clbm_net_get_params(self._h, _addr(t)), "clbm_net_get_params")
        return t

    def grads(self):
        import torch
        t = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check(lib().clbm_net_get_grads(self._h, _addr(t)), "clbm_net_get_grads")
        return t

    def forward(self, x):
        import torch
        x = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        assert tuple(x.shape) == self.shape_in, (x.shape, self.shape_in)
        y = torch.empty(self.shape_out, dtype=torch.float32, device=self.device)
        _check(lib().clbm_net_forward(self._h, _addr(x), _addr(y)), "clbm_net_forward")
        self._keep_x = x
        return y

    def backward(self, target):
        import torch
        t = torch.as_tensor(target, dtype=torch.float32, device=self.device).contiguous()
        assert tuple(t.shape) == self.shape_out
        loss = ctypes.c_double()
        _check(lib().clbm_net_backward(self._h, _addr(t), ctypes.byref(loss)), "clbm_net_backward")
        return loss.value

    def adam(self, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().clbm_net_adam(self._h, float(lr), float(beta1), float(beta2), float(eps), int(t)),
               "clbm_net_adam")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().clbm_net_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def resample(src, dh, dw, scale=None, shift=None, stream=None):
    """Bilinear resampling of float32 fields [nf][sh][sw] (device tensor) to [nf][dh][dw],
    field f scaled by scale[f] and shifted by shift[f]."""
    import torch
    src = src.contiguous()
    nf, sh, sw = src.shape
    dst = torch.empty(nf, int(dh), int(dw), dtype=torch.float32, device=src.device)
    sc = (ctypes.c_float * nf)(*scale) if scale is not None else None
    sf = (ctypes.c_float * nf)(*shift) if shift is not None else None
    _check(lib().clbm_resample_bilinear(_addr(src), sh, sw, _addr(dst), int(dh), int(dw), nf, sc, sf,
                                        _stream_ptr(stream)), "clbm_resample_bilinear")
    return dst


def problem_code(prob):
    """clbm_problem_code of a problem dict (computed by the library)."""
    c = clbm_problem_code()
    _check(lib().clbm_problem_encode(ctypes.byref(make_params(prob)), ctypes.byref(c)),
           "clbm_problem_encode")
    return c


def features(codes, height, width, device="cuda", stream=None):
    """Network input planes [len(codes)][8][height][width] from problem codes (device kernel)."""
    import torch
    raw = bytes((clbm_problem_code * len(codes))(*codes))
    d_codes = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
    out = torch.empty(len(codes), 8, int(height), int(width), dtype=torch.float32, device=device)
    _check(lib().clbm_net_features(_addr(d_codes), len(codes), int(height), int(width), _addr(out),
                                   _stream_ptr(stream)), "clbm_net_features")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    return out


def nusselt(diag, side, H, dT, into_wall=True):
    """Average Nusselt number at one wall from the mean outward gradient of Eq. (27).
    into_wall=True: heat flowing from the fluid into the wall (a cold wall),
    -dT/dn * H/dT; into_wall=False: heat entering the fluid (a hot wall)."""
    q = -diag.dTdn[side] * H / dT
    return q if into_wall else -q


def nusselt_flux(diag, side, H, dT, alpha, into_wall=True):
    """The same Nusselt number from the heat carried by the bounced links (wall_flux):
    wall_flux * H/(alpha dT). Agrees with nusselt() up to the discretisation error."""
    q = diag.wall_flux[side] * H / (alpha * dT)
    return q if into_wall else -q
