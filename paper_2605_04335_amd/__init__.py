"""Python binding of libibmpoisson (MI355X / gfx950).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels.  PyTorch provides device memory (tensors) and streams.  The
library must have been built (``python -m paper_2605_04335_amd.build`` or
``__graft_entry__.build()``); importing this module fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibmpoisson.so")

IBM_OK, IBM_EINVAL, IBM_EGEOM, IBM_ENOMEM, IBM_EHIP, IBM_ENOCONV, IBM_EBREAKDOWN, IBM_EAGAIN, IBM_ENOTFOUND = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
PREC_FP64, PREC_MIXED = 0, 1
PRECOND_MG, PRECOND_SRJ = 0, 1
SRJ_MAX_SWEEPS = 16
IBM_REQ_QUEUED, IBM_REQ_RUNNING, IBM_REQ_DONE, IBM_REQ_FAILED = 0, 1, 2, 3
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)


class IbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("xf", _c_double_p), ("yf", _c_double_p), ("zf", _c_double_p)]


class _Body(ctypes.Structure):
    _fields_ = [("n_vert", ctypes.c_int32), ("n_tri", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("vert", _c_double_p), ("tri", _c_int32_p)]


class _ClassStats(ctypes.Structure):
    _fields_ = [("n_solid", ctypes.c_int64), ("n_ghost", ctypes.c_int64), ("n_mghost", ctypes.c_int64),
                ("n_cut_links", ctypes.c_int64), ("pin", ctypes.c_int64)]


class PoissonOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("coarse_sweeps", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("srj_sweeps", ctypes.c_int32)]


BC_NEUMANN, BC_DIRICHLET = 0, 1


class AdOpts(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("tol", ctypes.c_double), ("sweeps", ctypes.c_int32),
                ("max_cycles", ctypes.c_int32)]


class AdStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("solve_ms", ctypes.c_double)]


class PoissonStats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("outer_steps", ctypes.c_int32), ("status", ctypes.c_int32),
                ("levels", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("pin_residual", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("n_fallback", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("device", ctypes.c_int32),
                ("cache_entries", ctypes.c_int32)]


class _Request(ctypes.Structure):
    _fields_ = [("grid", _Grid), ("bodies", ctypes.POINTER(_Body)), ("n_body", ctypes.c_int32),
                ("f", _c_double_p), ("opts", PoissonOpts)]


class ReqTimes(ctypes.Structure):
    _fields_ = [("submit_ms", ctypes.c_double), ("admit_ms", ctypes.c_double), ("done_ms", ctypes.c_double),
                ("n_unknowns", ctypes.c_int64), ("cache_hit", ctypes.c_int32), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]


EXPORTS = ["ibm_classify", "ibm_build_ghost_stencils", "ibm_stencils_info", "ibm_stencils_export",
           "ibm_stencils_free", "poisson_default_opts", "poisson_setup", "poisson_workspace_estimate",
           "poisson_solve", "poisson_apply", "poisson_assemble_rhs", "poisson_precond", "poisson_solve_assembled",
           "poisson_destroy", "poisson_workspace_size", "poisson_bind_workspace", "poisson_server_create",
           "poisson_submit", "poisson_poll", "poisson_server_drain", "poisson_server_destroy", "ibm_last_error",
           "poisson_update", "poisson_solve_from", "ibm_fill_fresh", "ibm_surface_forces",
           "ibm_build_ghost_stencils_bc", "ibm_ad_default_opts", "ibm_ad_setup", "ibm_ad_apply", "ibm_ad_solve",
           "ibm_ad_destroy", "ibm_hbm_stream", "poisson_kernel_timing", "ibm_classify_noalloc"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libibmpoisson.so is not built (%s); run paper_2605_04335_amd/build.py" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        L.ibm_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "ibm_last_error" and hasattr(L, name):
                getattr(L, name).restype = ctypes.c_int32
        L.ibm_stencils_free.restype = None
        L.poisson_destroy.restype = None
        L.poisson_default_opts.restype = None
        if hasattr(L, "ibm_ad_default_opts"):
            L.ibm_ad_default_opts.restype = None
            L.ibm_ad_destroy.restype = None
        if hasattr(L, "poisson_server_destroy"):
            L.poisson_server_destroy.restype = None
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        msg = lib().ibm_last_error().decode(errors="replace")
        raise IbmError(rc, "%s: %s" % (what, msg))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_c_double_p)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _tptr(t):
    return ctypes.c_void_p(t.data_ptr())


class _GridArgs:
    def __init__(self, xf, yf, zf):
        self.arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (xf, yf, zf)]
        self.g = _Grid(len(self.arrs[0]) - 1, len(self.arrs[1]) - 1, len(self.arrs[2]) - 1,
                       _dptr(self.arrs[0]), _dptr(self.arrs[1]), _dptr(self.arrs[2]))

    @property
    def N(self):
        return self.g.nx * self.g.ny * self.g.nz


class _BodyArgs:
    def __init__(self, bodies):
        self.keep = []
        n = len(bodies)
        self.arr = (_Body * max(n, 1))()
        for i, b in enumerate(bodies):
            v = np.ascontiguousarray(b.verts, dtype=np.float64).ravel()
            t = np.ascontiguousarray(b.tris, dtype=np.int32).ravel()
            self.keep += [v, t]
            self.arr[i] = _Body(len(v) // 3, len(t) // 3, int(b.kind), _dptr(v), t.ctypes.data_as(_c_int32_p))
        self.n = n


def default_opts(**kw) -> PoissonOpts:
    o = PoissonOpts()
    lib().poisson_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PREC_MIXED if v == "mixed" else PREC_FP64
        if k == "precond" and isinstance(v, str):
            v = PRECOND_SRJ if v == "srj" else PRECOND_MG
        setattr(o, k, v)
    return o


STREAM_COPY, STREAM_TRIAD, STREAM_READ = 0, 1, 2


def hbm_stream(kind: int, nbytes: int, reps: int = 10):
    """Streaming bandwidth of the device (ibm_hbm_stream): (GB/s, ms per
    pass, bytes read plus written per pass)."""
    ms = ctypes.c_double()
    moved = ctypes.c_double()
    _check(lib().ibm_hbm_stream(ctypes.c_int32(kind), ctypes.c_size_t(nbytes), ctypes.c_int32(reps),
                                ctypes.byref(ms), ctypes.byref(moved), _stream()), "ibm_hbm_stream")
    return moved.value / (ms.value * 1e-3) / 1e9, ms.value, moved.value


KERNEL_SWEEP0, KERNEL_APPLY0, KERNEL_XR = 0, 1, 2


# ------------------------------------------------------------------ geometry
def classify(xf, yf, zf, bodies, device="cuda"):
    """Device uint8 flags (torch) and counts."""
    import torch
    G = _GridArgs(xf, yf, zf)
    B = _BodyArgs(bodies)
    flags = torch.empty(G.N, dtype=torch.uint8, device=device)
    st = _ClassStats()
    _check(lib().ibm_classify(ctypes.byref(G.g), B.arr, ctypes.c_int32(B.n), _tptr(flags), ctypes.byref(st),
                              _stream()), "ibm_classify")
    return flags, {k: getattr(st, k) for k, _ in st._fields_}


CLASSIFY_NOALLOC_MAX_BYTES = 64 << 20


def classify_noalloc(xf, yf, zf, bodies, flags=None):
    """ibm_classify_noalloc: the classification with every device buffer of
    the call in the library's fixed per-device array (no device allocation
    in the library).  flags: a device uint8 tensor of N cells to write
    (allocated here when None).  Returns (flags, counts, scratch bytes)."""
    import torch
    G = _GridArgs(xf, yf, zf)
    B = _BodyArgs(bodies)
    if flags is None:
        flags = torch.empty(G.N, dtype=torch.uint8, device="cuda")
    assert flags.dtype == torch.uint8 and flags.is_cuda and flags.numel() >= G.N
    st = _ClassStats()
    need = ctypes.c_size_t()
    _check(lib().ibm_classify_noalloc(ctypes.byref(G.g), B.arr, ctypes.c_int32(B.n), _tptr(flags), ctypes.byref(st),
                                      ctypes.byref(need), _stream()), "ibm_classify_noalloc")
    return flags, {k: getattr(st, k) for k, _ in st._fields_}, need.value


def fill_fresh(xf, yf, zf, flags_old, flags_new, x) -> int:
    """Fresh cells (fluid now, solid before) take the mean of their neighbours
    that are fluid at both steps; x (device double[N]) in place.  Returns the
    fresh-cell count."""
    G = _GridArgs(xf, yf, zf)
    n = ctypes.c_int64()
    _check(lib().ibm_fill_fresh(ctypes.byref(G.g), _tptr(flags_old), _tptr(flags_new), _tptr(x), ctypes.byref(n),
                                _stream()), "ibm_fill_fresh")
    return n.value


def surface_forces(xf, yf, zf, bodies, flags, p):
    """Nodal pressure forces (device double[total vertices, 3], body by
    body), per-triangle pressure jumps (device double[total triangles]) and
    the count of probes with no usable interpolation node."""
    import torch
    G = _GridArgs(xf, yf, zf)
    B = _BodyArgs(bodies)
    nv = sum(len(b.verts) for b in bodies)
    nt = sum(len(b.tris) for b in bodies)
    F = torch.zeros((max(nv, 1), 3), dtype=torch.float64, device=p.device)
    dp = torch.zeros(max(nt, 1), dtype=torch.float64, device=p.device)
    lost = ctypes.c_int64()
    _check(lib().ibm_surface_forces(ctypes.byref(G.g), B.arr, ctypes.c_int32(B.n), _tptr(flags), _tptr(p), _tptr(F),
                                    _tptr(dp), ctypes.byref(lost), _stream()), "ibm_surface_forces")
    return F[:nv], dp[:nt], lost.value


class Stencils:
    def __init__(self, handle, N):
        self.h = handle
        self.N = N

    def info(self):
        ng, nm, nf = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ibm_stencils_info(self.h, ctypes.byref(ng), ctypes.byref(nm), ctypes.byref(nf)), "info")
        return ng.value, nm.value, nf.value

    def export(self):
        ng, nm, nf = self.info()
        rows = ng + nm
        out = dict(cell=np.zeros(rows, np.int32), col=np.zeros((rows, 8), np.int32), w=np.zeros((rows, 8)),
                   sG=np.zeros(rows), dlb=np.zeros(rows), rfl=np.zeros(rows, np.uint8), geo=np.zeros((rows, 12)))
        if rows:
            _check(lib().ibm_stencils_export(self.h, out["cell"].ctypes.data_as(_c_int32_p),
                                             out["col"].ctypes.data_as(_c_int32_p), _dptr(out["w"]),
                                             _dptr(out["sG"]), _dptr(out["dlb"]),
                                             out["rfl"].ctypes.data_as(ctypes.c_void_p), _dptr(out["geo"])),
                   "export")
        out["ng"], out["nm"], out["nfallback"] = ng, nm, nf
        return out

    def close(self):
        if self.h:
            lib().ibm_stencils_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_ghost_stencils(xf, yf, zf, bodies, flags, bc: str = "neumann") -> Stencils:
    """Ghost rows: Neumann (pressure) or Dirichlet (advection-diffusion)."""
    G = _GridArgs(xf, yf, zf)
    B = _BodyArgs(bodies)
    h = ctypes.c_void_p()
    code = {"neumann": BC_NEUMANN, "dirichlet": BC_DIRICHLET}[bc]
    _check(lib().ibm_build_ghost_stencils_bc(ctypes.byref(G.g), B.arr, ctypes.c_int32(B.n), _tptr(flags),
                                             ctypes.c_int32(code), ctypes.byref(h), _stream()),
           "ibm_build_ghost_stencils_bc")
    return Stencils(h, G.N)


# ------------------------------------------------------------------ advection-diffusion step
class AdSolver:
    """An ibm_ad_ctx: H u = u - beta L u with Dirichlet ghost rows, solved by SRJ cycles."""

    def __init__(self, xf, yf, zf, flags, stencils: "Stencils", beta: float, tol: float = 1e-10, sweeps: int = 8,
                 max_cycles: int = 500):
        self.G = _GridArgs(xf, yf, zf)
        o = AdOpts()
        lib().ibm_ad_default_opts(ctypes.byref(o))
        o.beta, o.tol, o.sweeps, o.max_cycles = beta, tol, sweeps, max_cycles
        self.opts = o
        ng, nm, nf = stencils.info()
        self.N, self.nm, self.ng = self.G.N, nm, ng
        self.h = ctypes.c_void_p()
        _check(lib().ibm_ad_setup(ctypes.byref(self.G.g), _tptr(flags), stencils.h, ctypes.byref(o),
                                  ctypes.byref(self.h)), "ibm_ad_setup")

    def _vec(self, device="cuda"):
        import torch
        return torch.zeros(self.N + self.nm, dtype=torch.float64, device=device)

    def apply(self, x, y=None):
        if y is None:
            y = self._vec(x.device)
        _check(lib().ibm_ad_apply(self.h, _tptr(x), _tptr(y), _stream()), "ibm_ad_apply")
        return y

    def solve(self, f, g=None, u=None, check=True):
        """u (device double[N + n_mghost]) is the initial guess and receives the solution."""
        if u is None:
            u = self._vec(f.device)
        st = AdStats()
        rc = lib().ibm_ad_solve(self.h, _tptr(f), _tptr(g) if g is not None else None, _tptr(u), ctypes.byref(st),
                                _stream())
        if check:
            _check(rc, "ibm_ad_solve")
        return u, st

    def close(self):
        if self.h:
            lib().ibm_ad_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ solver
class Solver:
    """A poisson_ctx: level-0 operator, multigrid hierarchy and work vectors."""

    def __init__(self, xf, yf, zf, flags, stencils: Stencils, opts: Optional[PoissonOpts] = None, **kw):
        self.G = _GridArgs(xf, yf, zf)
        self.opts = opts if opts is not None else default_opts(**kw)
        ng, nm, nf = stencils.info()
        self.N, self.nm, self.ng = self.G.N, nm, ng
        self.h = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        _check(lib().poisson_setup(ctypes.byref(self.G.g), _tptr(flags), stencils.h, ctypes.byref(self.opts),
                                   ctypes.byref(nbytes), ctypes.byref(self.h)), "poisson_setup")
        self.workspace_bytes = nbytes.value

    @property
    def n_unknowns(self):
        return self.N + self.nm

    def kernel_timing(self, kernel: int, reset: bool = True):
        """Select a kernel for per-launch HIP-event timing in the following
        solves (-1: off); returns (total ms, launches) accumulated so far."""
        tot = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().poisson_kernel_timing(self.h, ctypes.c_int32(kernel), ctypes.c_int32(1 if reset else 0),
                                           ctypes.byref(tot), ctypes.byref(cnt)), "poisson_kernel_timing")
        return tot.value, cnt.value


    def _vec(self, device="cuda"):
        import torch
        return torch.zeros(self.n_unknowns, dtype=torch.float64, device=device)

    def solve(self, f, g=None, x=None, check=True):
        import torch
        assert f.dtype == torch.float64 and f.is_cuda and f.is_contiguous() and f.numel() == self.N
        if x is None:
            x = self._vec(f.device)
        st = PoissonStats()
        rc = lib().poisson_solve(self.h, _tptr(f), _tptr(g) if g is not None else None, _tptr(x),
                                 ctypes.byref(st), _stream())
        if check:
            _check(rc, "poisson_solve")
        return x, st

    def solve_from(self, f, x0, g=None, x=None, check=True):
        """Solve from an initial guess x0 (device double[N] cell values, or
        double[N + n_mghost] with the membrane ghost values)."""
        import torch
        assert f.dtype == torch.float64 and f.is_cuda and f.is_contiguous() and f.numel() == self.N
        assert x0.dtype == torch.float64 and x0.is_cuda and x0.is_contiguous()
        if x is None:
            x = self._vec(f.device)
        st = PoissonStats()
        rc = lib().poisson_solve_from(self.h, _tptr(f), _tptr(g) if g is not None else None, _tptr(x0),
                                      ctypes.c_int64(x0.numel()), _tptr(x), ctypes.byref(st), _stream())
        if check:
            _check(rc, "poisson_solve_from")
        return x, st

    def update(self, flags, stencils: "Stencils"):
        """Re-set-up for moved bodies: same grid and options, new flags and ghost rows."""
        _check(lib().poisson_update(self.h, _tptr(flags), stencils.h), "poisson_update")
        ng, nm, nf = stencils.info()
        self.nm, self.ng = nm, ng

    def solve_assembled(self, b, x=None, check=True):
        if x is None:
            x = self._vec(b.device)
        st = PoissonStats()
        rc = lib().poisson_solve_assembled(self.h, _tptr(b), _tptr(x), ctypes.byref(st), _stream())
        if check:
            _check(rc, "poisson_solve_assembled")
        return x, st

    def workspace_size(self) -> int:
        """Bytes of per-call scratch that bind_workspace can place in caller memory."""
        b = ctypes.c_size_t()
        _check(lib().poisson_workspace_size(self.h, ctypes.byref(b)), "poisson_workspace_size")
        return b.value

    def bind_workspace(self, ws):
        """Place the scratch in a caller-owned device tensor (kept referenced here)."""
        _check(lib().poisson_bind_workspace(self.h, ctypes.c_void_p(ws.data_ptr()),
                                            ctypes.c_size_t(ws.numel() * ws.element_size())),
               "poisson_bind_workspace")
        self._ws = ws

    def apply(self, x, y=None):
        if y is None:
            y = self._vec(x.device)
        _check(lib().poisson_apply(self.h, _tptr(x), _tptr(y), _stream()), "poisson_apply")
        return y

    def precond(self, b, x=None):
        if x is None:
            x = self._vec(b.device)
        _check(lib().poisson_precond(self.h, _tptr(b), _tptr(x), _stream()), "poisson_precond")
        return x

    def assemble_rhs(self, f, g=None, b=None):
        if b is None:
            b = self._vec(f.device)
        _check(lib().poisson_assemble_rhs(self.h, _tptr(f), _tptr(g) if g is not None else None, _tptr(b),
                                          _stream()), "poisson_assemble_rhs")
        return b

    def close(self):
        if self.h:
            lib().poisson_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_estimate(nx, ny, nz, n_rows, precision=PREC_FP64) -> int:
    if isinstance(precision, str):
        precision = PREC_MIXED if precision == "mixed" else PREC_FP64
    b = ctypes.c_size_t()
    _check(lib().poisson_workspace_estimate(nx, ny, nz, ctypes.c_int64(n_rows), precision, ctypes.byref(b)),
           "poisson_workspace_estimate")
    return b.value


def setup(xf, yf, zf, bodies, **opts):
    """classify + ghost stencils + solver setup for one problem."""
    flags, cst = classify(xf, yf, zf, bodies)
    st = build_ghost_stencils(xf, yf, zf, bodies, flags)
    sol = Solver(xf, yf, zf, flags, st, **opts)
    return flags, st, sol, cst


# ------------------------------------------------------------------ serving
class Server:
    """Persistent continuous-batching solve server (one device)."""

    def __init__(self, hbm_budget: int, max_slots: int = 16, device: int = 0, cache_entries: int = 8):
        self.h = ctypes.c_void_p()
        self._cells = {}
        o = _ServerOpts(hbm_budget, max_slots, device, cache_entries)
        _check(lib().poisson_server_create(ctypes.byref(o), ctypes.byref(self.h)), "poisson_server_create")

    def submit(self, xf, yf, zf, bodies, f, opts: Optional[PoissonOpts] = None, **kw) -> int:
        G = _GridArgs(xf, yf, zf)
        B = _BodyArgs(bodies)
        ff = np.ascontiguousarray(f, dtype=np.float64)
        req = _Request(G.g, ctypes.cast(B.arr, ctypes.POINTER(_Body)), B.n, _dptr(ff),
                       opts if opts is not None else default_opts(**kw))
        t = ctypes.c_uint64()
        _check(lib().poisson_submit(self.h, ctypes.byref(req), ctypes.byref(t)), "poisson_submit")
        self._cells[t.value] = (len(xf) - 1) * (len(yf) - 1) * (len(zf) - 1)
        return t.value

    def poll(self, ticket: int, want_x: bool = True):
        """(rc, state, x or None, stats, times); rc IBM_EAGAIN while unfinished.
        A finished request is consumed by the call that returns it."""
        n = self._cells.get(ticket, 0) if want_x else 0
        while True:
            x = np.zeros(max(n, 1))
            st = PoissonStats()
            tm = ReqTimes()
            state = ctypes.c_int32()
            rc = lib().poisson_poll(self.h, ctypes.c_uint64(ticket), _dptr(x) if n else None, ctypes.c_int64(n),
                                    ctypes.byref(st), ctypes.byref(tm), ctypes.byref(state))
            if rc == IBM_EINVAL and n and tm.n_unknowns > n:
                n = tm.n_unknowns  # membrane ghost unknowns follow the cells
                continue
            if rc != IBM_EAGAIN:
                self._cells.pop(ticket, None)
            return rc, state.value, (x[:tm.n_unknowns] if n else None), st, tm

    def drain(self):
        _check(lib().poisson_server_drain(self.h), "poisson_server_drain")

    def close(self):
        if self.h:
            lib().poisson_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
