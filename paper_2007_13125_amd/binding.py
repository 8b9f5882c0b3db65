"""Thin ctypes binding of the C ABI in ``include/pint.h``.

Argument marshalling only: every step of a sweep runs in the HIP kernels of
``libpint.so``.  PyTorch provides device memory and the stream.  The library
must have been built (``python -m paper_2007_13125_amd.build``); there is no
fallback path, and a missing library raises immediately.
"""
import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_longlong, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpint.so")

PINT_OK = 0
PINT_NOT_CONVERGED = 1
PINT_E_ARG = -1
PINT_E_UNSUPPORTED = -2
PINT_E_NOMEM = -3
PINT_E_HIP = -4
PINT_E_DIVERGED = -5

PRECISION = {"fp64": 0, "mixed": 1}
FORM = {"residual": 0, "direct": 1}
NORM = {"inf": 0, "l2T": 1}
INIT = {"v": 0, "zero": 1, "user": 2}
SPACE = {"fd": 0, "fem": 1}


class pint_grid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("m", c_int * 3), ("len", c_double * 3)]


class pint_params(ctypes.Structure):
    _fields_ = [("k", c_int), ("alpha", c_double), ("T", c_double), ("N", c_int),
                ("kappa", c_double), ("tol", c_double), ("max_sweeps", c_int),
                ("precision", c_int), ("form", c_int), ("norm", c_int), ("init", c_int), ("space", c_int)]


EXPORTS = {
    "pint_plan_create": (c_int, [POINTER(c_void_p), POINTER(pint_grid), POINTER(pint_params), c_void_p]),
    "pint_plan_workspace_bytes": (c_size_t, [c_void_p]),
    "pint_plan_set_workspace": (c_int, [c_void_p, c_void_p, c_size_t]),
    "pint_bind": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "pint_init_iterate": (c_int, [c_void_p, c_void_p]),
    "pint_sweeps": (c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    "pint_profile_sweeps": (c_int, [c_void_p, c_void_p, c_int, POINTER(c_double),
                                    POINTER(ctypes.c_char_p), c_int]),
    "pint_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                           POINTER(c_double), POINTER(c_double), POINTER(c_int)]),
    "pint_solve_windows": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, POINTER(c_double),
                                   POINTER(c_int)]),
    "pint_sequential_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "pint_nonlinear_solve": (c_int, [c_void_p, c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                     c_double, POINTER(c_int), POINTER(c_double), POINTER(c_int)]),
    "pint_solve_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                   POINTER(c_double), POINTER(c_double), POINTER(c_int)]),
    "pint_batch_plan_create": (c_int, [POINTER(c_void_p), c_int, POINTER(pint_grid),
                                       POINTER(pint_params), c_void_p]),
    "pint_batch_solve": (c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                 POINTER(c_void_p), POINTER(c_double), c_int, POINTER(c_int)]),
    "pint_plan_set_autotune": (c_int, [c_void_p, c_int]),
    "pint_plan_tune": (c_int, [c_void_p, c_void_p, c_int]),
    "pint_plan_get_variants": (c_int, [c_void_p, c_int, POINTER(c_int)]),
    "pint_plan_set_variants": (c_int, [c_void_p, c_int, POINTER(c_int)]),
    "pint_plan_destroy": (c_int, [c_void_p]),
    "pint_plan_unknowns": (c_longlong, [c_void_p]),
    "pint_status_str": (ctypes.c_char_p, [c_int]),
    "pint_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libpint.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2007_13125_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PintError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        L = lib()
        msg = L.pint_last_error().decode()
        super().__init__(f"{where}: {L.pint_status_str(status).decode()} ({msg})")


def _check(status, where, allow=(PINT_OK,)):
    if status not in allow:
        raise PintError(status, where)
    return status


def make_grid(m, length=None):
    g = pint_grid()
    g.dim = len(m)
    for i in range(3):
        g.m[i] = int(m[i]) if i < len(m) else 1
        g.len[i] = float(length[i]) if (length and i < len(length)) else 1.0
    return g


def make_params(k, alpha, T, N, kappa, tol=1e-12, max_sweeps=50, precision="fp64", form="residual",
                norm="inf", init="v", space="fd"):
    p = pint_params()
    p.k, p.alpha, p.T, p.N, p.kappa = int(k), float(alpha), float(T), int(N), float(kappa)
    p.tol, p.max_sweeps = float(tol), int(max_sweeps)
    p.precision, p.form, p.norm, p.init = PRECISION[precision], FORM[form], NORM[norm], INIT[init]
    p.space = SPACE[space]
    return p


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


# --- entry points under their C names ---------------------------------------------------

def pint_plan_create(grid, params, stream=None):
    """Returns a plan handle (c_void_p); stream is a torch.cuda.Stream or None (current stream)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    h = c_void_p()
    _check(lib().pint_plan_create(ctypes.byref(h), ctypes.byref(grid), ctypes.byref(params),
                                  c_void_p(stream.cuda_stream)), "pint_plan_create")
    return h


def pint_plan_workspace_bytes(plan):
    return int(lib().pint_plan_workspace_bytes(plan))


def pint_plan_set_workspace(plan, ws):
    _check(lib().pint_plan_set_workspace(plan, _ptr(ws), ws.numel() * ws.element_size()),
           "pint_plan_set_workspace")


def pint_bind(plan, v, f=None, fder=None):
    _check(lib().pint_bind(plan, _ptr(v), _ptr(f), _ptr(fder)), "pint_bind")


def pint_init_iterate(plan, U):
    _check(lib().pint_init_iterate(plan, _ptr(U)), "pint_init_iterate")


def pint_sweeps(plan, U, nsweeps, dev_norms=None):
    _check(lib().pint_sweeps(plan, _ptr(U), int(nsweeps), _ptr(dev_norms)), "pint_sweeps")


def pint_profile_sweeps(plan, U, nsweeps, max_slots=16):
    """Returns [(slot name, average ms per sweep)] measured with HIP events."""
    ms = (c_double * max_slots)()
    names = (ctypes.c_char_p * max_slots)()
    n = lib().pint_profile_sweeps(plan, _ptr(U), int(nsweeps), ms, names, max_slots)
    if n < 0:
        raise PintError(n, "pint_profile_sweeps")
    return [(names[i].decode(), ms[i]) for i in range(min(n, max_slots))]


def pint_solve(plan, v, f, fder, U, max_sweeps):
    """Returns (status, upd[max_sweeps], upd_l2T[max_sweeps], sweeps)."""
    upd = (c_double * max_sweeps)()
    upd2 = (c_double * max_sweeps)()
    nsw = c_int(0)
    st = lib().pint_solve(plan, _ptr(v), _ptr(f), _ptr(fder), _ptr(U), upd, upd2, ctypes.byref(nsw))
    _check(st, "pint_solve", allow=(PINT_OK, PINT_NOT_CONVERGED, PINT_E_DIVERGED))
    n = nsw.value
    return st, list(upd)[:n], list(upd2)[:n], n


def pint_solve_windows(plan, nwin, v, f, fder, U, max_sweeps):
    """Returns (status, per-window update norms, per-window sweep counts)."""
    upd = (c_double * (nwin * max_sweeps))()
    sw = (c_int * nwin)()
    st = lib().pint_solve_windows(plan, int(nwin), _ptr(v), _ptr(f), _ptr(fder), _ptr(U), upd, sw)
    _check(st, "pint_solve_windows", allow=(PINT_OK, PINT_NOT_CONVERGED))
    sw = list(sw)
    return st, [list(upd)[i * max_sweeps:i * max_sweeps + sw[i]] for i in range(nwin)], sw


def pint_sequential_solve(plan, v, f, fder, U):
    _check(lib().pint_sequential_solve(plan, _ptr(v), _ptr(f), _ptr(fder), _ptr(U)), "pint_sequential_solve")


def pint_nonlinear_solve(plan, c3, c1, v, f, fder, U, newton_steps, newton_tol=0.0):
    """Algorithm 3 for d^alpha u + A u + c3 u^3 + c1 u = f.  Returns (status,
    inner sweep counts, max |W_l| per Newton step)."""
    inner = (c_int * newton_steps)()
    upd = (c_double * newton_steps)()
    n = c_int(0)
    st = lib().pint_nonlinear_solve(plan, float(c3), float(c1), _ptr(v), _ptr(f), _ptr(fder), _ptr(U),
                                    int(newton_steps), float(newton_tol), inner, upd, ctypes.byref(n))
    _check(st, "pint_nonlinear_solve", allow=(PINT_OK, PINT_NOT_CONVERGED))
    return st, list(inner)[:n.value], list(upd)[:n.value]


def pint_solve_noalloc(plan, v, f, fder, U, max_sweeps):
    """pint_solve with the workspace in the library's static device array (no
    allocation).  Returns (status, upd, upd_l2T, sweeps); errors come back as the
    status, not raised (PINT_E_ARG for a plan whose workspace exceeds the array)."""
    upd = (c_double * max_sweeps)()
    upd2 = (c_double * max_sweeps)()
    nsw = c_int(0)
    st = lib().pint_solve_noalloc(plan, _ptr(v), _ptr(f), _ptr(fder), _ptr(U), upd, upd2, ctypes.byref(nsw))
    n = nsw.value
    return st, list(upd)[:n], list(upd2)[:n], n


def pint_batch_plan_create(grids, params, stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    n = len(grids)
    G = (pint_grid * n)(*grids)
    Pm = (pint_params * n)(*params)
    h = c_void_p()
    _check(lib().pint_batch_plan_create(ctypes.byref(h), n, G, Pm, c_void_p(stream.cuda_stream)),
           "pint_batch_plan_create")
    return h


def pint_batch_solve(plan, v, f, fder, U, max_sweeps):
    """max_sweeps: the row stride of the update-norm buffer; the library rejects
    it (PINT_E_ARG) if an instance may sweep more often.  Returns (status,
    per-instance update norms, per-instance sweep counts)."""
    n = len(v)
    arr = lambda ts: (c_void_p * n)(*[None if t is None else t.data_ptr() for t in ts])
    upd = (c_double * (n * max_sweeps))()
    sw = (c_int * n)()
    st = lib().pint_batch_solve(plan, arr(v), arr(f), arr(fder), arr(U), upd, int(max_sweeps), sw)
    _check(st, "pint_batch_solve", allow=(PINT_OK, PINT_NOT_CONVERGED, PINT_E_DIVERGED))
    sw = list(sw)
    u = list(upd)
    return st, [u[i * max_sweeps:i * max_sweeps + sw[i]] for i in range(n)], sw


def pint_plan_set_autotune(plan, reps):
    _check(lib().pint_plan_set_autotune(plan, int(reps)), "pint_plan_set_autotune")


def pint_plan_tune(plan, U, reps):
    _check(lib().pint_plan_tune(plan, _ptr(U), int(reps)), "pint_plan_tune")


def pint_plan_get_variants(plan, instance=0):
    """The kernel variants in use: [forward, x pass, y/z pass, 1D tridiagonal split]."""
    c = (c_int * 4)()
    _check(lib().pint_plan_get_variants(plan, int(instance), c), "pint_plan_get_variants")
    return list(c)


def pint_plan_set_variants(plan, choices, instance=0):
    c = (c_int * 4)(*[int(x) for x in choices])
    _check(lib().pint_plan_set_variants(plan, int(instance), c), "pint_plan_set_variants")


def pint_plan_destroy(plan):
    lib().pint_plan_destroy(plan)


def pint_plan_unknowns(plan):
    return int(lib().pint_plan_unknowns(plan))


# --- convenience wrapper ------------------------------------------------------------------

class Plan:
    """One problem on one device: owns the plan handle and a torch-allocated workspace."""

    def __init__(self, m, k, alpha, T, N, kappa, tol=1e-12, max_sweeps=50, precision="fp64",
                 form="residual", norm="inf", init="v", length=None, stream=None, space="fd"):
        import torch
        self.m, self.N, self.max_sweeps = tuple(m), int(N), int(max_sweeps)
        self.M = 1
        for x in m:
            self.M *= int(x)
        self.grid = make_grid(m, length)
        self.params = make_params(k, alpha, T, N, kappa, tol, max_sweeps, precision, form, norm, init, space)
        self.h = pint_plan_create(self.grid, self.params, stream)
        nbytes = pint_plan_workspace_bytes(self.h)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        off = (-self.ws.data_ptr()) % 256
        self._ws_view = self.ws[off:off + nbytes]
        pint_plan_set_workspace(self.h, self._ws_view)

    def bind(self, v, f=None, fder=None):
        self._data = (v, f, fder)       # keep the tensors alive while bound
        pint_bind(self.h, v, f, fder)

    def init_iterate(self, U):
        pint_init_iterate(self.h, U)

    def sweeps(self, U, n, dev_norms=None):
        pint_sweeps(self.h, U, n, dev_norms)

    def profile(self, U, n):
        return pint_profile_sweeps(self.h, U, n)

    def set_autotune(self, reps):
        pint_plan_set_autotune(self.h, reps)

    def tune(self, U, reps=3):
        pint_plan_tune(self.h, U, reps)
        return self.variants()

    def variants(self):
        return pint_plan_get_variants(self.h, 0)

    def set_variants(self, choices):
        pint_plan_set_variants(self.h, choices, 0)

    def solve(self, v, f=None, fder=None, U=None):
        import torch
        if U is None:
            U = torch.empty((self.N, self.M), dtype=torch.float64, device="cuda")
        self._data = (v, f, fder)
        st, upd, upd2, n = pint_solve(self.h, v, f, fder, U, self.max_sweeps)
        return U, {"status": st, "upd": upd, "upd_l2T": upd2, "sweeps": n}

    def close(self):
        if self.h is not None:
            pint_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
