"""Python binding of ``libfuglbm.so`` (the C ABI in ``include/fuglbm.h``).

Argument marshalling only: every step of the update runs in the HIP kernels.
PyTorch provides device memory (a uint8 tensor handed to ``fl_create_ext``) and
the HIP stream.  Importing this module does not need a GPU; creating a solver
does, and fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfuglbm.so")

FL_OK, FL_EINVAL, FL_EDOMAIN, FL_ENOMEM, FL_EDEVICE, FL_ENUMERIC, FL_ENOTCONV, FL_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6, -7
FL_MAX_COMP = 4
EOS = {"PR": 0, "SRK": 1, "VDW": 2}
LATTICE = {"D2Q9": 0, "D3Q19": 1}
COLLISION = {"BGK": 0, "MRT": 1}
PRECISION = {"fp64": 0, "fp32": 1}
FORCE_MODEL = {"wb": 0, "standard": 1}
STENCIL = {"axis": 0, "isotropic": 1}


class FLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fuglbm status {status}: {msg}")
        self.status = status


class fl_component(C.Structure):
    _fields_ = [("Tc", C.c_double), ("Pc", C.c_double), ("omega", C.c_double),
                ("M", C.c_double), ("kappa", C.c_double)]


class fl_params(C.Structure):
    _fields_ = [
        ("ncomp", C.c_int), ("comp", C.POINTER(fl_component)), ("kij", C.POINTER(C.c_double)),
        ("T", C.c_double), ("R", C.c_double), ("eos", C.c_int), ("lattice", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("collision", C.c_int),
        ("tau", C.c_double), ("mrt_rates", C.POINTER(C.c_double)), ("precision", C.c_int),
        ("force_time_level", C.c_int), ("force_model", C.c_int), ("stencil", C.c_int),
    ]


_lib = None
_DP = C.POINTER(C.c_double)
_VP = C.c_void_p

# name -> (restype, argtypes); mirrors include/fuglbm.h
SIGNATURES = {
    "fl_validate": (C.c_int, [C.POINTER(fl_params)]),
    "fl_required_bytes": (C.c_int, [C.POINTER(fl_params), C.POINTER(C.c_size_t)]),
    "fl_create": (C.c_int, [C.POINTER(fl_params), C.POINTER(_VP)]),
    "fl_create_ext": (C.c_int, [C.POINTER(fl_params), _VP, C.c_size_t, _VP, C.POINTER(_VP)]),
    "fl_destroy": (None, [_VP]),
    "fl_set_tuning": (C.c_int, [_VP, C.c_char_p]),
    "fl_last_error": (C.c_char_p, [_VP]),
    "fl_status_string": (C.c_char_p, [C.c_int]),
    "fl_lattice_table": (C.c_int, [C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), _DP]),
    "fl_set_state": (C.c_int, [_VP, _DP, _DP]),
    "fl_step": (C.c_int, [_VP, C.c_long]),
    "fl_step_timed": (C.c_int, [_VP, C.c_long, _DP, C.POINTER(C.c_char_p), C.POINTER(C.c_int)]),
    "fl_step_timed_every": (C.c_int, [_VP, C.c_long, C.c_long, _DP, C.POINTER(C.c_char_p), C.POINTER(C.c_int),
                                      C.POINTER(C.c_long)]),
    "fl_steps_done": (C.c_long, [_VP]),
    "fl_get_fields": (C.c_int, [_VP, _DP, _DP, _DP, _DP]),
    "fl_get_populations": (C.c_int, [_VP, _DP]),
    "fl_mass": (C.c_int, [_VP, _DP]),
    "fl_run_until": (C.c_int, [_VP, C.c_double, C.c_long, C.c_long, C.POINTER(C.c_long), _DP]),
    "fl_state_bytes": (C.c_int, [_VP, C.POINTER(C.c_size_t)]),
    "fl_get_state_raw": (C.c_int, [_VP, _VP, C.c_size_t]),
    "fl_set_state_raw": (C.c_int, [_VP, _VP, C.c_size_t]),
    "fl_server_create": (C.c_int, [C.POINTER(fl_params), C.c_size_t, C.c_int, _VP, C.POINTER(_VP)]),
    "fl_server_destroy": (None, [_VP]),
    "fl_server_set_tuning": (C.c_int, [_VP, C.c_char_p]),
    "fl_server_last_error": (C.c_char_p, [_VP]),
    "fl_server_request_bytes": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_size_t)]),
    "fl_server_submit": (C.c_int, [_VP, C.c_int, C.c_int, C.c_int, _DP, C.c_double, C.c_long, C.c_long,
                                   C.POINTER(C.c_uint64)]),
    "fl_server_tick": (C.c_int, [_VP, C.c_long, C.c_double, C.POINTER(C.c_int)]),
    "fl_server_poll": (C.c_int, [_VP, C.POINTER(C.c_uint64), C.c_int, C.POINTER(C.c_int)]),
    "fl_server_result": (C.c_int, [_VP, C.c_uint64, _DP, _DP, _DP, C.POINTER(C.c_long), _DP, C.POINTER(C.c_int),
                                   _DP]),
    "fl_server_result_noalloc": (C.c_int, [_VP, C.c_uint64, _DP, _DP, _DP, C.POINTER(C.c_long), _DP,
                                           C.POINTER(C.c_int), _DP]),
    "fl_server_info": (C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_size_t),
                                 C.POINTER(C.c_size_t)]),
}


def load():
    """Load the built library; raises ImportError when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run python -m paper_2212_10680_amd.build")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_DP)


class Params:
    """Owns the ctypes fl_params and the arrays it points to."""

    def __init__(self, components, T, shape, lattice="D2Q9", kij=None, R=1.0, eos="PR",
                 collision="BGK", tau=1.0, mrt_rates=None, precision="fp64", force_time_level=0,
                 force_model="wb", stencil="axis"):
        nc = len(components)
        self._args = dict(components=[dict(c) for c in components], T=T, lattice=lattice, kij=kij, R=R,
                          eos=eos, collision=collision, tau=tau, mrt_rates=mrt_rates,
                          precision=precision, force_time_level=force_time_level, force_model=force_model,
                          stencil=stencil)
        self._comp = (fl_component * nc)(*[fl_component(c["Tc"], c["Pc"], c["omega"], c["M"], c["kappa"])
                                           for c in components])
        self._kij = None
        if kij is not None:
            self._kij = np.ascontiguousarray(np.asarray(kij, dtype=np.float64).reshape(nc * nc))
        self._mrt = None
        if mrt_rates is not None:
            self._mrt = np.ascontiguousarray(np.asarray(mrt_rates, dtype=np.float64))
        shape = tuple(int(s) for s in shape)
        if len(shape) == 2:
            shape = shape + (1,)
        self.shape = shape
        self.ncomp = nc
        self.lattice = lattice
        self.D = 2 if lattice == "D2Q9" else 3
        self.Q = 9 if lattice == "D2Q9" else 19
        self.N = shape[0] * shape[1] * shape[2]
        self.precision = precision
        p = fl_params()
        p.ncomp = nc
        p.comp = C.cast(self._comp, C.POINTER(fl_component))
        p.kij = _dp(self._kij)
        p.T, p.R = float(T), float(R)
        p.eos = EOS[eos]
        p.lattice = LATTICE[lattice]
        p.nx, p.ny, p.nz = shape
        p.collision = COLLISION[collision]
        p.tau = float(tau)
        p.mrt_rates = _dp(self._mrt)
        p.precision = PRECISION[precision]
        p.force_time_level = int(force_time_level)
        p.force_model = FORCE_MODEL[force_model]
        p.stencil = STENCIL[stencil]
        self.c = p

    @classmethod
    def from_workload(cls, w, precision=None, shape=None, **kw):
        comps, kij, T = w.thermo()
        kw.setdefault("eos", w.eos)
        return cls(comps, T, shape or w.shape, lattice=w.lattice, kij=kij, collision=w.collision,
                   tau=w.tau, precision=precision or w.precision, **kw)

    def with_shape(self, shape, precision=None):
        """Same problem on another lattice shape (and optionally precision)."""
        kw = dict(self._args)
        if precision is not None:
            kw["precision"] = precision
        comps, T = kw.pop("components"), kw.pop("T")
        return Params(comps, T, shape, **kw)

    def validate(self):
        return load().fl_validate(C.byref(self.c))

    def required_bytes(self):
        n = C.c_size_t(0)
        st = load().fl_required_bytes(C.byref(self.c), C.byref(n))
        if st != FL_OK:
            raise FLError(st, "invalid parameters")
        return n.value


def lattice_table(lattice):
    lib = load()
    q = C.c_int(0)
    e = (C.c_int * (19 * 3))()
    w = np.zeros(19)
    st = lib.fl_lattice_table(LATTICE[lattice], C.byref(q), e, _dp(w))
    if st != FL_OK:
        raise FLError(st, "lattice")
    Q = q.value
    return np.array(e[:3 * Q]).reshape(Q, 3), w[:Q]


class Solver:
    """A solver on torch-owned device memory and the current torch stream."""

    def __init__(self, params: Params, device="cuda"):
        import torch  # device memory and streams only

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the fuglbm solver runs only on the HIP device")
        lib = load()
        self.p = params
        self.lib = lib
        nbytes = params.required_bytes()
        self.mem = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.mem.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = torch.cuda.current_stream(device)
        h = _VP()
        st = lib.fl_create_ext(C.byref(params.c), C.c_void_p(aligned), C.c_size_t(nbytes),
                               C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != FL_OK:
            raise FLError(st, "fl_create_ext failed")
        self.h = h

    def _check(self, st, what):
        if st != FL_OK:
            msg = self.lib.fl_last_error(self.h)
            raise FLError(st, f"{what}: {msg.decode() if msg else ''}")
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.fl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- calls
    def set_tuning(self, spec=None):
        """Launch tuning on top of the measured defaults (fl_set_tuning)."""
        arg = None if spec is None else spec.encode()
        self._check(self.lib.fl_set_tuning(self.h, arg), "fl_set_tuning")

    def set_state(self, rho_molar, u=None):
        p = self.p
        r = np.ascontiguousarray(np.asarray(rho_molar, dtype=np.float64).reshape(p.ncomp, p.N))
        uu = None if u is None else np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(p.D, p.N))
        self._check(self.lib.fl_set_state(self.h, _dp(r), _dp(uu)), "fl_set_state")

    def step(self, n):
        return self._check(self.lib.fl_step(self.h, int(n)), "fl_step")

    def step_timed_every(self, n, every):
        """Advance n steps, timing the kernels of every `every`-th one; returns
        ({kernel name: mean ms per launch over the timed steps}, timed steps)."""
        ms = np.zeros(8)
        names = (C.c_char_p * 8)()
        k = C.c_int(8)
        t = C.c_long(0)
        self._check(self.lib.fl_step_timed_every(self.h, int(n), int(every), _dp(ms), names, C.byref(k),
                                                 C.byref(t)), "fl_step_timed_every")
        return {names[i].decode(): ms[i] / max(t.value, 1) for i in range(k.value)}, t.value

    def step_timed(self, n):
        ms = np.zeros(8)
        names = (C.c_char_p * 8)()
        k = C.c_int(8)
        self._check(self.lib.fl_step_timed(self.h, int(n), _dp(ms), names, C.byref(k)), "fl_step_timed")
        return {names[i].decode(): ms[i] for i in range(k.value)}

    @property
    def steps(self):
        return self.lib.fl_steps_done(self.h)

    def fields(self):
        p = self.p
        out = {"rho_molar": np.zeros((p.ncomp, p.N)), "u": np.zeros((p.D, p.N)), "p": np.zeros(p.N),
               "lnf": np.zeros((p.ncomp, p.N))}
        self._check(self.lib.fl_get_fields(self.h, _dp(out["rho_molar"]), _dp(out["u"]), _dp(out["p"]),
                                           _dp(out["lnf"])), "fl_get_fields")
        return out

    def populations(self):
        p = self.p
        g = np.zeros((p.ncomp, p.Q, p.N))
        self._check(self.lib.fl_get_populations(self.h, _dp(g)), "fl_get_populations")
        return g

    def mass(self):
        m = np.zeros(self.p.ncomp)
        self._check(self.lib.fl_mass(self.h, _dp(m)), "fl_mass")
        return m

    def run_until(self, tol, check_every, max_steps):
        done = C.c_long(0)
        res = C.c_double(0.0)
        st = self.lib.fl_run_until(self.h, float(tol), int(check_every), int(max_steps), C.byref(done),
                                   C.byref(res))
        if st not in (FL_OK, FL_ENOTCONV):
            self._check(st, "fl_run_until")
        return st == FL_OK, done.value, res.value

    def get_state_raw(self):
        n = C.c_size_t(0)
        self._check(self.lib.fl_state_bytes(self.h, C.byref(n)), "fl_state_bytes")
        buf = np.zeros(n.value, dtype=np.uint8)
        self._check(self.lib.fl_get_state_raw(self.h, buf.ctypes.data_as(_VP), n), "fl_get_state_raw")
        return buf

    def set_state_raw(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.fl_set_state_raw(self.h, buf.ctypes.data_as(_VP), C.c_size_t(buf.size)),
                    "fl_set_state_raw")


class Server:
    """Batched server (fl_server_*): many independent lattices, one batched
    kernel launch per tick.  The server owns its pool of device memory."""

    def __init__(self, params: Params, pool_bytes, max_slots=512):
        import torch  # the current torch stream carries the server's work

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the fuglbm server runs only on the HIP device")
        self.lib = load()
        self.p = params
        self.stream = torch.cuda.current_stream()
        h = _VP()
        st = self.lib.fl_server_create(C.byref(params.c), C.c_size_t(int(pool_bytes)), int(max_slots),
                                       C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if st != FL_OK:
            raise FLError(st, "fl_server_create failed")
        self.h = h

    def _check(self, st, what):
        if st not in (FL_OK,):
            msg = self.lib.fl_server_last_error(self.h)
            raise FLError(st, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None):
            self.lib.fl_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, spec=None):
        """Server launch tuning (fl_server_set_tuning): serve, serve_cap, serve_group."""
        arg = None if spec is None else spec.encode()
        self._check(self.lib.fl_server_set_tuning(self.h, arg), "fl_server_set_tuning")

    def request_bytes(self, shape):
        nx, ny, nz = (tuple(shape) + (1,))[:3]
        b = C.c_size_t(0)
        self._check(self.lib.fl_server_request_bytes(self.h, nx, ny, nz, C.byref(b)), "request_bytes")
        return b.value

    def submit(self, rho_molar, shape, tol, check_every, max_steps):
        """Returns the request id, or None when the server cannot admit it now."""
        nx, ny, nz = (tuple(shape) + (1,))[:3]
        r = np.ascontiguousarray(np.asarray(rho_molar, dtype=np.float64).reshape(self.p.ncomp, -1))
        rid = C.c_uint64(0)
        st = self.lib.fl_server_submit(self.h, nx, ny, nz, _dp(r), float(tol), int(check_every),
                                       int(max_steps), C.byref(rid))
        if st == FL_EAGAIN:
            return None
        self._check(st, "fl_server_submit")
        return rid.value

    def tick(self, steps, max_ms=0.0):
        """Advance the running requests (oldest first, at most as many as the
        device holds server workgroups at once) by up to `steps` steps or
        max_ms of device time (<= 0: no limit); returns the number still
        running."""
        a = C.c_int(0)
        self._check(self.lib.fl_server_tick(self.h, int(steps), float(max_ms), C.byref(a)), "fl_server_tick")
        return a.value

    def poll(self, cap=4096):
        ids = (C.c_uint64 * cap)()
        n = C.c_int(0)
        self._check(self.lib.fl_server_poll(self.h, ids, cap, C.byref(n)), "fl_server_poll")
        return [ids[i] for i in range(n.value)]

    def result(self, rid, n_nodes, full=False):
        """Collect a finished request: (rho_molar, steps, residual, status), or
        with full=True a dict that adds u, p and latency_s."""
        rho = np.zeros((self.p.ncomp, n_nodes))
        u = np.zeros((self.p.D, n_nodes)) if full else None
        pr = np.zeros(n_nodes) if full else None
        steps = C.c_long(0)
        res = C.c_double(0.0)
        status = C.c_int(0)
        lat = C.c_double(0.0)
        self._check(self.lib.fl_server_result(self.h, C.c_uint64(rid), _dp(rho), _dp(u), _dp(pr), C.byref(steps),
                                              C.byref(res), C.byref(status), C.byref(lat)), "fl_server_result")
        if full:
            return {"rho_molar": rho, "u": u, "p": pr, "steps": steps.value, "residual": res.value,
                    "status": status.value, "latency_s": lat.value}
        return rho, steps.value, res.value, status.value

    def info(self):
        a, f = C.c_int(0), C.c_int(0)
        used, tot = C.c_size_t(0), C.c_size_t(0)
        self._check(self.lib.fl_server_info(self.h, C.byref(a), C.byref(f), C.byref(used), C.byref(tot)),
                    "fl_server_info")
        return {"active": a.value, "free_slots": f.value, "pool_used": used.value, "pool_total": tot.value}
