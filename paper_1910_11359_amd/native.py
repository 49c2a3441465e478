"""ctypes binding of libipeps.so (argument marshalling only).

Every call below forwards to the C ABI declared in include/ipeps.h; no step
of the method runs in Python.  Loading fails loudly when the gfx950 library
has not been built (``python -m paper_1910_11359_amd.build``).
"""
import ctypes as C
import weakref
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libipeps.so")

IPEPS_OK = 0
IPEPS_EINVAL = -1
IPEPS_ENOMEM = -2
IPEPS_EDEVICE = -3
IPEPS_ENUMERIC = -4
IPEPS_ENOTCONV = -5
IPEPS_EAGAIN = -6
IPEPS_ENOTFOUND = -7
IPEPS_ETOOBIG = -8
DTYPES = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
FLAG_AUTOTUNE = 1
FLAG_FACTORED_CUTS = 2
FLAG_FORMED_CUTS = 4
JOB_QUEUED, JOB_RUNNING, JOB_DONE = 0, 1, 2


class Config(C.Structure):
    _fields_ = [("D", C.c_int), ("chi", C.c_int), ("d_A", C.c_int),
                ("J", C.c_double), ("V", C.c_double), ("W", C.c_double), ("dt", C.c_double),
                ("trotter_order", C.c_int), ("dtype", C.c_int),
                ("layer_J", C.c_double * 4), ("layer_V", C.c_double * 4),
                ("layer_w", C.c_double * 4), ("flags", C.c_uint32), ("seed", C.c_uint64)]


class Obs(C.Structure):
    _fields_ = [("t", C.c_double), ("n", C.c_double * 4), ("imbalance", C.c_double),
                ("sum_n", C.c_double), ("max_offdiag", C.c_double),
                ("trunc_err", C.c_double * 4), ("ctm_iters", C.c_int), ("ctm_delta", C.c_double),
                ("renyi1", C.c_double * 4), ("renyi_half", C.c_double * 4)]

    def as_dict(self):
        return {"t": self.t, "n": np.array(self.n[:]), "imbalance": self.imbalance,
                "sum_n": self.sum_n, "max_offdiag": self.max_offdiag,
                "eps": np.array(self.trunc_err[:]), "ctm_iters": self.ctm_iters,
                "ctm_delta": self.ctm_delta, "renyi1": np.array(self.renyi1[:]),
                "renyi_half": np.array(self.renyi_half[:])}


class Job(C.Structure):
    _fields_ = [("cfg", Config), ("n_steps", C.c_int), ("observe_every", C.c_int),
                ("ctm_iters", C.c_int), ("tag", C.c_uint64)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)

EXPORTS = [
    "ipeps_config_default", "ipeps_footprint_bytes", "ipeps_init", "ipeps_set_state",
    "ipeps_get_state", "ipeps_trotter_step", "ctmrg_converge", "ipeps_observe",
    "ipeps_corner_spectra", "ipeps_bond_spectra", "ipeps_destroy", "solve_server_create",
    "solve_submit", "solve_poll", "solve_job_times", "solve_server_destroy", "ipeps_strerror",
    "ipeps_profile", "ipeps_profile_read", "ff_neel_dynamics", "ff_bessel_j",
    "ipeps_observe_async", "ipeps_observe_result", "ff_spectrum_ipr", "ff_neel_dynamics_noalloc",
    "ipeps_profile_read_gemms", "ipeps_slab_region_bytes", "ipeps_slab_create", "ipeps_slab_init",
    "ipeps_slab_destroy", "ipeps_batch_create", "ipeps_batch_trotter_step", "ipeps_batch_ctmrg",
    "ipeps_batch_observe", "ipeps_batch_destroy", "ipeps_batch_observe_async", "ipeps_batch_query",
    "ipeps_batch_observe_result", "ipeps_batch_set_graph", "solve_server_set_graphs",
]

_lib = None


def load():
    """Load libipeps.so once; raises if it is missing or incomplete."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run python -m paper_1910_11359_amd.build")
    lib = C.CDLL(LIB_PATH)
    for name in EXPORTS:
        if not hasattr(lib, name):
            raise ImportError(f"libipeps.so lacks {name}")
    P = C.POINTER
    lib.ipeps_config_default.argtypes = [P(Config)]
    lib.ipeps_config_default.restype = None
    lib.ipeps_footprint_bytes.argtypes = [P(Config)]
    lib.ipeps_footprint_bytes.restype = C.c_size_t
    lib.ipeps_init.argtypes = [P(Config), C.c_void_p, ALLOC_FN, FREE_FN, C.c_void_p, P(C.c_void_p)]
    lib.ipeps_set_state.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.ipeps_get_state.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
    lib.ipeps_trotter_step.argtypes = [C.c_void_p, C.c_int, P(C.c_double)]
    lib.ctmrg_converge.argtypes = [C.c_void_p, C.c_double, C.c_int, C.c_int, P(C.c_int),
                                   P(C.c_double)]
    lib.ipeps_observe.argtypes = [C.c_void_p, P(Obs)]
    lib.ipeps_observe_async.argtypes = [C.c_void_p]
    lib.ipeps_observe_result.argtypes = [C.c_void_p, P(Obs)]
    lib.ipeps_corner_spectra.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ipeps_bond_spectra.argtypes = [C.c_void_p, P(C.c_double)]
    lib.ipeps_destroy.argtypes = [C.c_void_p]
    lib.ipeps_destroy.restype = None
    lib.solve_server_create.argtypes = [C.c_size_t, C.c_int, P(C.c_void_p)]
    lib.solve_submit.argtypes = [C.c_void_p, P(Job), P(C.c_uint64)]
    lib.solve_poll.argtypes = [C.c_void_p, C.c_uint64, P(C.c_int), P(Obs), C.c_int, P(C.c_int)]
    lib.solve_job_times.argtypes = [C.c_void_p, C.c_uint64, P(C.c_double), P(C.c_double),
                                    P(C.c_double)]
    lib.solve_server_set_graphs.argtypes = [C.c_void_p, C.c_int]
    lib.solve_server_destroy.argtypes = [C.c_void_p]
    lib.solve_server_destroy.restype = None
    lib.ipeps_profile.argtypes = [C.c_void_p, C.c_int]
    lib.ipeps_profile_read.argtypes = [C.c_void_p, P(C.c_double), P(C.c_int), P(C.c_double)]
    lib.ipeps_profile_read_gemms.argtypes = [C.c_void_p, C.c_int, P(C.c_double), P(C.c_double), P(C.c_double),
                                             P(C.c_int)]
    lib.ff_neel_dynamics.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int,
                                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.ff_neel_dynamics_noalloc.argtypes = lib.ff_neel_dynamics.argtypes
    lib.ff_bessel_j.argtypes = [C.c_double, C.c_int, P(C.c_double)]
    lib.ff_spectrum_ipr.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.ipeps_slab_region_bytes.argtypes = [P(Config)]
    lib.ipeps_slab_region_bytes.restype = C.c_size_t
    lib.ipeps_slab_create.argtypes = [P(Config), C.c_int, P(C.c_void_p)]
    lib.ipeps_slab_init.argtypes = [C.c_void_p, C.c_int, P(Config), C.c_void_p, P(C.c_void_p)]
    lib.ipeps_slab_destroy.argtypes = [C.c_void_p]
    lib.ipeps_slab_destroy.restype = None
    lib.ipeps_batch_create.argtypes = [P(C.c_void_p), C.c_int, P(C.c_void_p)]
    lib.ipeps_batch_trotter_step.argtypes = [C.c_void_p, C.c_int]
    lib.ipeps_batch_ctmrg.argtypes = [C.c_void_p, C.c_int, C.c_int]
    lib.ipeps_batch_set_graph.argtypes = [C.c_void_p, C.c_int]
    lib.ipeps_batch_observe.argtypes = [C.c_void_p, P(Obs)]
    lib.ipeps_batch_observe_async.argtypes = [C.c_void_p]
    lib.ipeps_batch_query.argtypes = [C.c_void_p]
    lib.ipeps_batch_observe_result.argtypes = [C.c_void_p, P(Obs), P(C.c_int)]
    lib.ipeps_batch_destroy.argtypes = [C.c_void_p]
    lib.ipeps_batch_destroy.restype = None
    lib.ipeps_strerror.argtypes = [C.c_int]
    lib.ipeps_strerror.restype = C.c_char_p
    _lib = lib
    return lib


class IpepsError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = load().ipeps_strerror(code).decode()
        super().__init__(f"{where}: {msg} ({code})")


def _check(code, where):
    if code != IPEPS_OK:
        raise IpepsError(code, where)


def make_config(D, chi, J=1.0, V=1.0, W=5.0, dt=0.05, d_A=2, dtype="fp64", layer_J=None,
                layer_V=None, layer_w=None, seed=1, flags=0):
    lib = load()
    c = Config()
    lib.ipeps_config_default(C.byref(c))
    c.D, c.chi, c.d_A = int(D), int(chi), int(d_A)
    c.J, c.V, c.W, c.dt = float(J), float(V), float(W), float(dt)
    c.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
    for name, val in (("layer_J", layer_J), ("layer_V", layer_V), ("layer_w", layer_w)):
        if val is not None:
            arr = getattr(c, name)
            for i in range(4):
                arr[i] = float(val[i])
    c.seed = int(seed)
    c.flags = int(flags)
    return c


def footprint_bytes(cfg):
    return int(load().ipeps_footprint_bytes(C.byref(cfg)))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class State:
    """One iPEPS job on the device (wraps ipeps_state*)."""

    def __init__(self, cfg, stream=None):
        lib = load()
        self.cfg = cfg
        self._lib = lib
        handle = C.c_void_p()
        sptr = None
        if stream is not None:  # a torch.cuda.Stream or a raw hipStream_t
            sptr = getattr(stream, "cuda_stream", stream)
        _check(lib.ipeps_init(C.byref(cfg), C.c_void_p(sptr), ALLOC_FN(), FREE_FN(), None,
                              C.byref(handle)), "ipeps_init")
        self.h = handle

    def close(self):
        """Destroys the state (a batch open over it is closed first)."""
        if getattr(self, "h", None):
            for b in list(getattr(self, "_batches", ())):
                b.close()
            self._lib.ipeps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, gamma, lam):
        g = np.ascontiguousarray(gamma, dtype=np.complex128).view(np.float64)
        l = np.ascontiguousarray(lam, dtype=np.float64)
        _check(self._lib.ipeps_set_state(self.h, _dptr(g), _dptr(l)), "ipeps_set_state")

    def get_state(self):
        D, d = self.cfg.D, 2 * self.cfg.d_A
        g = np.zeros((4, d, D, D, D, D), dtype=np.complex128)
        l = np.zeros((8, D))
        gv = g.view(np.float64)
        _check(self._lib.ipeps_get_state(self.h, _dptr(gv), _dptr(l)), "ipeps_get_state")
        return g, l

    def trotter_step(self, n_steps=1, want_eps=False):
        eps = np.zeros(4)
        _check(self._lib.ipeps_trotter_step(self.h, int(n_steps), _dptr(eps) if want_eps else None),
               "ipeps_trotter_step")
        return eps if want_eps else None

    def ctmrg(self, tol=0.0, max_iter=10, cold=True, allow_notconv=False, want_delta=True):
        it = C.c_int()
        dl = C.c_double()
        rc = self._lib.ctmrg_converge(self.h, float(tol), int(max_iter), int(bool(cold)),
                                      C.byref(it), C.byref(dl) if want_delta else None)
        if not (allow_notconv and rc == IPEPS_ENOTCONV):
            _check(rc, "ctmrg_converge")
        return it.value, (dl.value if want_delta else None)

    def observe(self):
        o = Obs()
        _check(self._lib.ipeps_observe(self.h, C.byref(o)), "ipeps_observe")
        return o.as_dict()

    def observe_async(self):
        """Start a readout of the current environment (result via observe_result)."""
        _check(self._lib.ipeps_observe_async(self.h), "ipeps_observe_async")

    def observe_result(self):
        o = Obs()
        _check(self._lib.ipeps_observe_result(self.h, C.byref(o)), "ipeps_observe_result")
        return o.as_dict()

    def corner_spectra(self):
        out = np.zeros((16, self.cfg.chi))
        _check(self._lib.ipeps_corner_spectra(self.h, _dptr(out)), "ipeps_corner_spectra")
        return out

    def profile(self, enable=True, every_gemm=False):
        mode = (2 if every_gemm else 1) if enable else 0
        _check(self._lib.ipeps_profile(self.h, mode), "ipeps_profile")

    def profile_read_gemms(self, dtype):
        """(summed ms, summed algorithmic flops, summed algorithmic bytes,
        launches) of the recorded GEMM launches whose arithmetic is dtype
        ('fp64', 'fp32', 'bf16', 'bf16x3')."""
        ms, fl, by, n = C.c_double(), C.c_double(), C.c_double(), C.c_int()
        _check(self._lib.ipeps_profile_read_gemms(self.h, DTYPES[dtype], C.byref(ms), C.byref(fl),
                                                  C.byref(by), C.byref(n)), "ipeps_profile_read_gemms")
        return ms.value, fl.value, by.value, n.value

    def profile_read(self):
        ms, n, fl = C.c_double(), C.c_int(), C.c_double()
        _check(self._lib.ipeps_profile_read(self.h, C.byref(ms), C.byref(n), C.byref(fl)),
               "ipeps_profile_read")
        return ms.value, n.value, fl.value

    def bond_spectra(self):
        out = np.zeros((8, self.cfg.D))
        _check(self._lib.ipeps_bond_spectra(self.h, _dptr(out)), "ipeps_bond_spectra")
        return out


class Slab:
    """One device allocation holding `slots` states of one layout
    (ipeps_slab_*; include/ipeps.h)."""

    def __init__(self, layout_cfg, slots):
        self._lib = load()
        h = C.c_void_p()
        _check(self._lib.ipeps_slab_create(C.byref(layout_cfg), int(slots), C.byref(h)), "ipeps_slab_create")
        self.h = h
        self._states = weakref.WeakSet()

    def state(self, slot, cfg, stream=None):
        st = State.__new__(State)
        st.cfg, st._lib = cfg, self._lib
        handle = C.c_void_p()
        sptr = getattr(stream, "cuda_stream", stream) if stream is not None else None
        _check(self._lib.ipeps_slab_init(self.h, int(slot), C.byref(cfg), C.c_void_p(sptr), C.byref(handle)),
               "ipeps_slab_init")
        st.h = handle
        st._slab = self  # the slab's memory outlives the state
        self._states.add(st)
        return st

    def close(self):
        """Destroys the states still open in the slab, then the slab."""
        if getattr(self, "h", None):
            for st in list(self._states):
                st.close()
            self._lib.ipeps_slab_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Lockstep batch of states of one slab (ipeps_batch_*); states[0] leads."""

    def __init__(self, states, graph=False):
        self._lib = load()
        self.states = list(states)
        arr = (C.c_void_p * len(self.states))(*[s.h.value for s in self.states])
        h = C.c_void_p()
        _check(self._lib.ipeps_batch_create(arr, len(self.states), C.byref(h)), "ipeps_batch_create")
        self.h = h
        for st in self.states:  # closing a state closes the batch first
            if not hasattr(st, "_batches"):
                st._batches = weakref.WeakSet()
            st._batches.add(self)
        if graph:
            self.set_graph(True)

    def set_graph(self, enable=True):
        """Replay the warm CTMRG iterations from a captured HIP graph."""
        _check(self._lib.ipeps_batch_set_graph(self.h, int(bool(enable))), "ipeps_batch_set_graph")

    def trotter_step(self, n_steps=1):
        _check(self._lib.ipeps_batch_trotter_step(self.h, int(n_steps)), "ipeps_batch_trotter_step")

    def ctmrg(self, iters, cold=True):
        _check(self._lib.ipeps_batch_ctmrg(self.h, int(iters), int(bool(cold))), "ipeps_batch_ctmrg")

    def observe(self):
        buf = (Obs * len(self.states))()
        _check(self._lib.ipeps_batch_observe(self.h, buf), "ipeps_batch_observe")
        return [buf[i].as_dict() for i in range(len(self.states))]

    def observe_status(self):
        """Readouts and per-job codes (a job whose readout is not finite gets
        IPEPS_ENUMERIC; the others' results stand)."""
        _check(self._lib.ipeps_batch_observe_async(self.h), "ipeps_batch_observe_async")
        buf = (Obs * len(self.states))()
        st = (C.c_int * len(self.states))()
        rc = self._lib.ipeps_batch_observe_result(self.h, buf, st)
        if rc not in (IPEPS_OK, IPEPS_ENUMERIC):
            _check(rc, "ipeps_batch_observe_result")
        return [buf[i].as_dict() for i in range(len(self.states))], list(st)

    def close(self):
        if getattr(self, "h", None):
            self._lib.ipeps_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """The request loop (wraps ipeps_server*)."""

    def __init__(self, hbm_budget=0, max_slots=4, graphs=False):
        self._lib = load()
        h = C.c_void_p()
        _check(self._lib.solve_server_create(C.c_size_t(int(hbm_budget)), int(max_slots),
                                             C.byref(h)), "solve_server_create")
        self.h = h
        if graphs:
            _check(self._lib.solve_server_set_graphs(self.h, 1), "solve_server_set_graphs")

    def submit(self, cfg, n_steps, observe_every=10, ctm_iters=10, tag=0):
        j = Job()
        j.cfg = cfg
        j.n_steps, j.observe_every, j.ctm_iters, j.tag = int(n_steps), int(observe_every), int(ctm_iters), int(tag)
        jid = C.c_uint64()
        _check(self._lib.solve_submit(self.h, C.byref(j), C.byref(jid)), "solve_submit")
        return jid.value

    def poll(self, job_id, cap=4096):
        status = C.c_int()
        n = C.c_int()
        buf = (Obs * cap)()
        rc = self._lib.solve_poll(self.h, C.c_uint64(job_id), C.byref(status), buf, cap, C.byref(n))
        if rc == IPEPS_EAGAIN:
            return status.value, None
        _check(rc, "solve_poll")
        return status.value, [buf[i].as_dict() for i in range(min(cap, n.value))]

    def times(self, job_id):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        rc = self._lib.solve_job_times(self.h, C.c_uint64(job_id), C.byref(a), C.byref(b), C.byref(c))
        return rc, (a.value, b.value, c.value)

    def close(self):
        if getattr(self, "h", None):
            self._lib.solve_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------- free-fermion dynamics
def ff_bessel_j(x, kmax):
    """J_0(x)..J_kmax(x) from the library's host copy of its coefficient routine."""
    out = np.zeros(kmax + 1)
    _check(load().ff_bessel_j(float(x), int(kmax), _dptr(out)), "ff_bessel_j")
    return out


def ff_neel_dynamics_device(L, eps_ptr, n_real, n_even_ptr, n_odd_ptr, n_times, dt, tau=0.5, pbc=False,
                            stream=None):
    """Enqueue on device buffers (raw pointers); see include/ff.h."""
    sptr = getattr(stream, "cuda_stream", stream) if stream is not None else None
    _check(load().ff_neel_dynamics(int(L), int(bool(pbc)), float(tau), float(dt), int(n_times), int(n_real),
                                   C.c_void_p(eps_ptr), C.c_void_p(n_even_ptr), C.c_void_p(n_odd_ptr),
                                   C.c_void_p(sptr)), "ff_neel_dynamics")


def ff_neel_dynamics_noalloc_device(L, eps_ptr, n_real, n_even_ptr, n_odd_ptr, n_times, dt, tau=0.5,
                                    pbc=False, stream=None):
    """The no-allocation variant (fixed device scratch; see include/ff.h)."""
    sptr = getattr(stream, "cuda_stream", stream) if stream is not None else None
    _check(load().ff_neel_dynamics_noalloc(int(L), int(bool(pbc)), float(tau), float(dt), int(n_times),
                                           int(n_real), C.c_void_p(eps_ptr), C.c_void_p(n_even_ptr),
                                           C.c_void_p(n_odd_ptr), C.c_void_p(sptr)),
           "ff_neel_dynamics_noalloc")


_hip = None


def _hip_runtime():
    """The HIP runtime libipeps.so itself links (not torch's bundled copy), for
    plain device buffers in the host convenience wrappers."""
    global _hip
    if _hip is None:
        load()
        h = C.CDLL("libamdhip64.so.7")
        h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        h.hipFree.argtypes = [C.c_void_p]
        h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        h.hipDeviceSynchronize.argtypes = []
        _hip = h
    return _hip


class _DeviceArray:
    """FP64 device buffer (hipMalloc / hipMemcpy of the library's runtime)."""

    H2D, D2H = 1, 2

    def __init__(self, n):
        self.n = int(n)
        self.p = C.c_void_p()
        if _hip_runtime().hipMalloc(C.byref(self.p), max(8, 8 * self.n)) != 0:
            raise IpepsError(IPEPS_ENOMEM, "hipMalloc")

    def put(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.size == self.n
        if _hip_runtime().hipMemcpy(self.p, a.ctypes.data, 8 * self.n, self.H2D) != 0:
            raise IpepsError(IPEPS_EDEVICE, "hipMemcpy")

    def get(self):
        out = np.empty(self.n)
        if self.n and _hip_runtime().hipMemcpy(out.ctypes.data, self.p, 8 * self.n, self.D2H) != 0:
            raise IpepsError(IPEPS_EDEVICE, "hipMemcpy")
        return out

    def get_int32(self):
        """The buffer's first 4 n bytes as int32 (the buffer holds 8 n)."""
        out = np.empty(self.n, dtype=np.int32)
        if self.n and _hip_runtime().hipMemcpy(out.ctypes.data, self.p, 4 * self.n, self.D2H) != 0:
            raise IpepsError(IPEPS_EDEVICE, "hipMemcpy")
        return out

    def __del__(self):
        if getattr(self, "p", None) and self.p.value:
            _hip_runtime().hipFree(self.p)
            self.p = C.c_void_p()


def ff_neel_dynamics(L, eps, n_times, dt, tau=0.5, pbc=False):
    """Host convenience: eps (n_real, L*L) -> (n_even, n_odd), each (n_real, n_times).
    Copies the fields to the device, runs on the default stream, copies back."""
    eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1, L * L)
    n_real = eps.shape[0]
    k = n_real * n_times
    d_eps, ne, no = _DeviceArray(eps.size), _DeviceArray(k), _DeviceArray(k)
    d_eps.put(eps)
    ff_neel_dynamics_device(L, d_eps.p.value, n_real, ne.p.value, no.p.value, n_times, dt, tau, pbc, None)
    if _hip_runtime().hipDeviceSynchronize() != 0:
        raise IpepsError(IPEPS_EDEVICE, "hipDeviceSynchronize")
    return ne.get().reshape(n_real, n_times), no.get().reshape(n_real, n_times)


def ff_spectrum_ipr_device(L, eps_ptr, n_real, e_ptr, ipr_ptr, bin_ptr, cnt_ptr, tau=0.5, pbc=False,
                           stream=None):
    """Enqueue on device buffers (raw pointers); see include/ff.h."""
    sptr = getattr(stream, "cuda_stream", stream) if stream is not None else None
    _check(load().ff_spectrum_ipr(int(L), int(bool(pbc)), float(tau), int(n_real), C.c_void_p(eps_ptr),
                                  C.c_void_p(e_ptr), C.c_void_p(ipr_ptr), C.c_void_p(bin_ptr),
                                  C.c_void_p(cnt_ptr), C.c_void_p(sptr)), "ff_spectrum_ipr")


def ff_spectrum_ipr(L, eps, tau=0.5, pbc=False):
    """Host convenience: eps (n_real, L*L) -> energies, ipr (n_real, L*L) and the
    per-bin IPR sums (n_real, 20) and state counts (n_real, 20, int32)."""
    eps = np.ascontiguousarray(eps, dtype=np.float64).reshape(-1, L * L)
    n_real, n = eps.shape
    d_eps, E, I = _DeviceArray(eps.size), _DeviceArray(n_real * n), _DeviceArray(n_real * n)
    B, K = _DeviceArray(n_real * 20), _DeviceArray(n_real * 20)
    d_eps.put(eps)
    ff_spectrum_ipr_device(L, d_eps.p.value, n_real, E.p.value, I.p.value, B.p.value, K.p.value, tau, pbc,
                           None)
    if _hip_runtime().hipDeviceSynchronize() != 0:
        raise IpepsError(IPEPS_EDEVICE, "hipDeviceSynchronize")
    return (E.get().reshape(n_real, n), I.get().reshape(n_real, n), B.get().reshape(n_real, 20),
            K.get_int32().reshape(n_real, 20))
