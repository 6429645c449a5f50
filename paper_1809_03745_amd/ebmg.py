"""ctypes binding of libebmg.so (include/ebmg.h). Argument marshalling only:
every step of setup and solve runs in the library (host C++ setup, HIP
kernels for the solve). The library must have been built
(``paper_1809_03745_amd.build``); importing this module fails loudly if it
is missing.

Device arrays are passed as torch tensors (their data_ptr on the context's
device); host arrays as numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libebmg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libebmg.so is not built: run `python -m paper_1809_03745_amd.build` "
                      "(or __graft_entry__.build()) first")

# One HIP runtime per process: torch ships its own libamdhip64 (same soname,
# different file). Loading torch first lets the library bind to that copy;
# loading the library first would bring in a second HIP/HSA runtime that sees
# no devices once torch initialises its own.
try:
    import torch as _torch  # noqa: F401
except ImportError:  # host-only use (setup and exports) needs no torch
    _torch = None

_lib = C.CDLL(LIB_PATH)

OK, ERR_ARG, ERR_GEOMETRY, ERR_OOM, ERR_DEVICE, ERR_NOCONV, ERR_NUMERIC, ERR_BUSY = range(8)
STATUS_NAMES = ["OK", "ERR_ARG", "ERR_GEOMETRY", "ERR_OOM", "ERR_DEVICE", "ERR_NOCONV", "ERR_NUMERIC",
                "ERR_BUSY"]
FP64, MIXED = 0, 1


class EbmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")
        self.status = status


class Box(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32 * 3), ("h", C.c_double), ("lo", C.c_double * 3)]


class Object(C.Structure):
    _fields_ = [("kind", C.c_int32), ("value", C.c_double), ("sdf", C.POINTER(C.c_double))]


class DomainBC(C.Structure):
    _fields_ = [("kind", C.c_int32 * 6), ("value", C.c_double * 6), ("robin_a1", C.c_double * 6),
                ("robin_a2", C.c_double * 6)]


class Options(C.Structure):
    _fields_ = [("alpha", C.c_double), ("beta", C.c_double), ("a_gas", C.c_double), ("a_diel", C.c_double),
                ("b_gas", C.c_double), ("dirichlet_closure", C.c_int32), ("robin_closure", C.c_int32),
                ("eb_order", C.c_int32), ("precision", C.c_int32), ("nu1", C.c_int32), ("nu2", C.c_int32),
                ("bottom_max_dof", C.c_int32), ("krylov", C.c_int32), ("smoother", C.c_int32),
                ("tail", C.c_int32), ("batch", C.c_int32), ("graphs", C.c_int32), ("reserved", C.c_int32 * 3)]


class SolveInfo(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("outer_iters", C.c_int32), ("levels", C.c_int32), ("n_hist", C.c_int32),
                ("r0_norm", C.c_double), ("rel_residual", C.c_double), ("seconds", C.c_double),
                ("est_bytes", C.c_int64), ("hist", C.c_double * 64)]

    def as_dict(self):
        return dict(cycles=self.cycles, outer_iters=self.outer_iters, levels=self.levels,
                    r0_norm=self.r0_norm, rel_residual=self.rel_residual, seconds=self.seconds,
                    est_bytes=self.est_bytes, hist=[self.hist[i] for i in range(self.n_hist)])


_vp = C.c_void_p
_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("ebmg_default_options", None, [C.POINTER(Options)])
_sig("ebmg_abi_version", C.c_int, [])
_sig("ebmg_create", C.c_int, [C.c_int32, _vp, C.POINTER(_vp)])
_sig("ebmg_destroy", C.c_int, [_vp])
_sig("ebmg_last_error", C.c_char_p, [_vp])
_sig("ebmg_setup", C.c_int, [_vp, C.POINTER(Box), C.c_int32, C.POINTER(Object), C.POINTER(DomainBC),
                             C.POINTER(Options), C.POINTER(_vp)])
_sig("ebmg_query", C.c_int, [_vp, _i64p, _i64p, C.POINTER(C.c_int32), _i64p])
_sig("ebmg_query_level", C.c_int, [_vp, C.c_int32, _i64p, _i64p])
_sig("ebmg_export_level", C.c_int, [_vp, C.c_int32, _vp, _vp, _vp])
_sig("ebmg_query_tuning", C.c_int, [_vp, C.c_int32, C.POINTER(C.c_int32), _dp, _dp])
_sig("ebmg_export_geometry", C.c_int, [_vp, _vp, _vp, _vp, _vp])
_sig("ebmg_export_moments", C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("ebmg_export_operator", C.c_int, [_vp, C.c_int32, _i64p, _vp, _vp, _vp])
_sig("ebmg_export_rhs", C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp])
_sig("ebmg_solve", C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_double, C.c_int32, _vp, _vp, _vp,
                             C.POINTER(SolveInfo)])
_sig("ebmg_submit", C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_double, C.c_int32, _vp, _vp, _vp,
                              C.POINTER(C.c_uint64)])
_sig("ebmg_poll", C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_int32), C.POINTER(C.c_int), C.POINTER(SolveInfo)])
_sig("ebmg_wait", C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_int), C.POINTER(SolveInfo)])
_sig("ebmg_apply", C.c_int, [_vp, _vp, _vp, _vp, _vp])
_sig("ebmg_apply_noalloc", C.c_int, [_vp, _vp, _vp, _vp, _vp])
_sig("ebmg_efield", C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("ebmg_time_kernel", C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _dp, _dp])
_sig("ebmg_smooth", C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _vp, _vp])
_sig("ebmg_restrict_residual", C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp])
_sig("ebmg_kernel_timing", C.c_int, [_vp, C.c_int32, C.c_int32, C.c_int32, _i64p, _dp, _dp])
_sig("ebmg_release", C.c_int, [_vp])
_sig("ebmg_set_coefficients", C.c_int, [_vp, C.POINTER(Options), C.POINTER(DomainBC)])
_sig("ebmg_setup_batch", C.c_int, [_vp, C.c_int32, C.POINTER(Box), C.POINTER(C.c_int32), C.POINTER(_vp),
                                   C.POINTER(DomainBC), C.POINTER(Options), C.POINTER(_vp)])
_sig("ebmg_query_batch", C.c_int, [_vp, _i64p, _i64p, _i64p])
_sig("ebmg_query_batch_box", C.c_int, [_vp, C.c_int32, _i64p, _i64p])
_sig("ebmg_query_batch_tuning", C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_double)])
_sig("ebmg_solve_batch", C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp), C.c_double, C.c_int32, C.POINTER(_vp),
                                   C.POINTER(_vp), C.POINTER(SolveInfo)])
_sig("ebmg_release_batch", C.c_int, [_vp])
_sig("ebmg_setup_family", C.c_int, [_vp, C.POINTER(Box), C.c_int32, C.POINTER(Object), C.c_int32, C.POINTER(DomainBC),
                                    C.POINTER(Options), C.POINTER(_vp)])
_sig("ebmg_query_family", C.c_int, [_vp, C.POINTER(C.c_int32), _i64p, _i64p, _i64p, _i64p])
_sig("ebmg_solve_family", C.c_int, [_vp, C.POINTER(_vp), C.POINTER(_vp), C.c_double, C.c_int32, C.POINTER(_vp),
                                    C.POINTER(_vp), C.POINTER(SolveInfo), C.POINTER(C.c_int)])
_sig("ebmg_release_family", C.c_int, [_vp])
_sig("ebmg_advect", C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_double, _vp, _vp])
_sig("ebmg_time_batch_kernel", C.c_int, [_vp, C.c_int32, C.c_int32, _vp, _vp])
_sig("ebmg_setup_amr", C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp])
_sig("ebmg_query_amr", C.c_int, [_vp, C.c_int32, _vp, _vp, _vp, _vp])
_sig("ebmg_solve_amr", C.c_int, [_vp, _vp, C.c_double, C.c_int32, _vp, _vp, _vp])
_sig("ebmg_apply_amr", C.c_int, [_vp, _vp, _vp, _vp, _vp])
_sig("ebmg_release_amr", C.c_int, [_vp])
_sig("ebmg_mesh_create", C.c_int, [_vp, C.c_int32, _vp, C.c_int32, _vp, C.POINTER(_vp)])
_sig("ebmg_mesh_query", C.c_int, [_vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32), _i64p])
_sig("ebmg_mesh_sdf", C.c_int, [_vp, C.POINTER(Box), _vp, _i64p])
_sig("ebmg_mesh_release", C.c_int, [_vp])

EXPORTED = ["ebmg_default_options", "ebmg_abi_version", "ebmg_create", "ebmg_destroy", "ebmg_last_error",
            "ebmg_setup", "ebmg_query", "ebmg_query_level", "ebmg_export_level", "ebmg_query_tuning",
            "ebmg_export_geometry", "ebmg_export_moments", "ebmg_export_operator", "ebmg_export_rhs",
            "ebmg_solve", "ebmg_submit", "ebmg_poll", "ebmg_wait", "ebmg_apply", "ebmg_apply_noalloc", "ebmg_efield", "ebmg_time_kernel", "ebmg_release",
            "ebmg_setup_batch", "ebmg_query_batch", "ebmg_query_batch_box", "ebmg_query_batch_tuning", "ebmg_solve_batch", "ebmg_release_batch",
            "ebmg_set_coefficients", "ebmg_smooth", "ebmg_restrict_residual", "ebmg_kernel_timing",
            "ebmg_setup_family", "ebmg_query_family", "ebmg_solve_family", "ebmg_release_family",
            "ebmg_mesh_create", "ebmg_mesh_query", "ebmg_mesh_sdf", "ebmg_mesh_release", "ebmg_advect",
            "ebmg_time_batch_kernel", "ebmg_setup_amr", "ebmg_query_amr", "ebmg_solve_amr", "ebmg_apply_amr", "ebmg_release_amr"]


def abi_version():
    return _lib.ebmg_abi_version()


def _ptr(a):
    """Address of a numpy array (host) or torch tensor (device); None -> NULL."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _host_f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _dev(ctx, t, n, name, nullable=False):
    """Device pointer of a float64 tensor argument, checked before the library
    sees it: a CPU, wrong-device, non-float64, non-contiguous or short tensor
    would be read or written out of bounds by the kernels, so it is refused
    here (EBMG_ERR_ARG) instead."""
    if t is None:
        if nullable:
            return None
        raise EbmgError(ERR_ARG, f"{name}: a device tensor is required")
    if _torch is None or not isinstance(t, _torch.Tensor):
        raise EbmgError(ERR_ARG, f"{name}: expected a torch tensor on cuda:{ctx.device}, got {type(t).__name__}")
    if not t.is_cuda or ctx.device < 0 or t.device.index != ctx.device:
        raise EbmgError(ERR_ARG, f"{name}: tensor on {t.device}, the context's device is cuda:{ctx.device}")
    if t.dtype != _torch.float64:
        raise EbmgError(ERR_ARG, f"{name}: dtype {t.dtype}, expected torch.float64")
    if not t.is_contiguous():
        raise EbmgError(ERR_ARG, f"{name}: tensor is not contiguous")
    if t.numel() < n:
        raise EbmgError(ERR_ARG, f"{name}: {t.numel()} elements, at least {n} needed")
    return t.data_ptr()


class Context:
    """A device (>= 0) with a HIP stream, or a host-only context (device < 0)."""

    def __init__(self, device=0, stream=None):
        h = _vp()
        st = _lib.ebmg_create(int(device), stream, C.byref(h))
        if st != OK:
            raise EbmgError(st, "ebmg_create failed: " + _lib.ebmg_last_error(None).decode(errors="replace"))
        self.h = h
        self.device = device
        self._held = {}  # ticket -> device tensors of a submitted solve

    def _collect(self, ticket, st, res, info):
        self.check(st, "ebmg_poll/ebmg_wait")
        self._held.pop(ticket, None)
        return res.value, info.as_dict()

    def poll(self, ticket):
        """None while the submitted solve ``ticket`` runs, else (status, info)."""
        done, res, info = C.c_int32(), C.c_int(), SolveInfo()
        st = _lib.ebmg_poll(self.h, C.c_uint64(ticket), C.byref(done), C.byref(res), C.byref(info))
        if st == OK and not done.value:
            return None
        return self._collect(ticket, st, res, info)

    def wait(self, ticket):
        """(status, info) of the submitted solve ``ticket``, blocking until it ends."""
        res, info = C.c_int(), SolveInfo()
        st = _lib.ebmg_wait(self.h, C.c_uint64(ticket), C.byref(res), C.byref(info))
        return self._collect(ticket, st, res, info)

    def check(self, st, what):
        if st != OK:
            msg = _lib.ebmg_last_error(self.h).decode(errors="replace")
            raise EbmgError(st, f"{what}: {msg}")

    def close(self):
        if self.h:
            _lib.ebmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


KRYLOV_AUTO, KRYLOV_NONE, KRYLOV_BICGSTAB = 0, 1, 2


def make_options(prob, precision=FP64, dirichlet_closure=0, robin_closure=0, eb_order=2, nu1=2, nu2=2,
                 bottom_max_dof=0, krylov=KRYLOV_AUTO, smoother=0, tail=0, batch=0, graphs=0):
    o = Options()
    _lib.ebmg_default_options(C.byref(o))
    o.alpha = prob.alpha
    o.beta = prob.beta
    o.a_gas = prob.a_gas
    o.a_diel = prob.a_diel
    o.b_gas = prob.b_gas
    o.dirichlet_closure = dirichlet_closure
    o.robin_closure = robin_closure
    o.eb_order = eb_order
    o.precision = precision
    o.nu1 = nu1
    o.nu2 = nu2
    o.bottom_max_dof = bottom_max_dof
    o.krylov = krylov
    o.smoother = smoother
    o.tail = tail
    o.batch = batch
    o.graphs = graphs
    return o


def _c_bc(prob):
    bc = DomainBC()
    for f in range(6):
        bc.kind[f] = prob.bc_kind[f]
        bc.value[f] = prob.bc_value[f]
        bc.robin_a1[f] = prob.robin_a1[f]
        bc.robin_a2[f] = prob.robin_a2[f]
    return bc


def _c_problem(prob):
    """(Box, Object array, DomainBC, kept SDF arrays) of a ``workloads.Problem``."""
    box = Box()
    box.dim = prob.dim
    for d in range(3):
        box.n[d] = prob.n[d] if d < prob.dim else 1
        box.lo[d] = prob.lo[d] if d < prob.dim else 0.0
    box.h = prob.h
    sdf = [np.ascontiguousarray(o.sdf, dtype=np.float64) for o in prob.objects]
    objs = (Object * max(1, len(prob.objects)))()
    for k, o in enumerate(prob.objects):
        objs[k].kind = o.kind
        objs[k].value = o.value
        objs[k].sdf = sdf[k].ctypes.data_as(_dp)
    bc = DomainBC()
    for f in range(6):
        bc.kind[f] = prob.bc_kind[f]
        bc.value[f] = prob.bc_value[f]
        bc.robin_a1[f] = prob.robin_a1[f]
        bc.robin_a2[f] = prob.robin_a2[f]
    return box, objs, bc, sdf


class Problem:
    """A problem set up in the library from a ``workloads.Problem``."""

    def __init__(self, ctx, prob, **opts):
        self.ctx = ctx
        self.prob = prob
        box, objs, bc, self._sdf = _c_problem(prob)
        self.options = make_options(prob, **opts)
        h = _vp()
        st = _lib.ebmg_setup(ctx.h, C.byref(box), len(prob.objects), objs, C.byref(bc), C.byref(self.options),
                             C.byref(h))
        self._sdf = None
        ctx.check(st, "ebmg_setup")
        self.h = h
        n, n2, lev, by = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int64()
        ctx.check(_lib.ebmg_query(h, C.byref(n), C.byref(n2), C.byref(lev), C.byref(by)), "ebmg_query")
        self.N, self.N2, self.levels, self.device_bytes = n.value, n2.value, lev.value, by.value

    # -- host exports ----------------------------------------------------------
    def geometry(self):
        kg = np.zeros(self.N)
        kd = np.zeros(self.N)
        pr = np.zeros(self.N, np.int8)
        sc = np.zeros(max(1, self.N2), np.int64)
        self.ctx.check(_lib.ebmg_export_geometry(self.h, _ptr(kg), _ptr(kd), _ptr(pr), _ptr(sc)),
                       "ebmg_export_geometry")
        return kg, kd, pr, sc[:self.N2]

    def moments(self, phase=0):
        """Cut-cell moments of one phase (host copies): dict of vcent
        (dim, N), apert (list of per-direction face arrays in numpy order),
        foff (list of (faces, dim-1) arrays), eb_area (N), eb_cent and
        eb_normal (dim, N)."""
        b = self.prob
        dim = b.dim
        n = list(b.n) + [1] * (3 - dim)
        counts = []
        shapes = []
        for d in range(dim):
            m = [n[e] + (1 if e == d else 0) for e in range(3)]
            counts.append(m[0] * m[1] * m[2])
            shapes.append(tuple(reversed(m[:dim])))
        F = sum(counts)
        vc = np.zeros(dim * self.N)
        ap = np.zeros(F)
        fo = np.zeros(max(1, (dim - 1) * F))
        ea = np.zeros(self.N)
        ec = np.zeros(dim * self.N)
        en = np.zeros(dim * self.N)
        self.ctx.check(_lib.ebmg_export_moments(self.h, int(phase), _ptr(vc), _ptr(ap), _ptr(fo), _ptr(ea), _ptr(ec),
                                                _ptr(en)), "ebmg_export_moments")
        aps, fos = [], []
        o = 0
        for d in range(dim):
            aps.append(ap[o:o + counts[d]].reshape(shapes[d]))
            fos.append(fo[(dim - 1) * o:(dim - 1) * (o + counts[d])].reshape(counts[d], dim - 1))
            o += counts[d]
        return dict(vcent=vc.reshape(dim, self.N), apert=aps, foff=fos, eb_area=ea,
                    eb_cent=ec.reshape(dim, self.N), eb_normal=en.reshape(dim, self.N))

    def level_size(self, level):
        n, n2 = C.c_int64(), C.c_int64()
        self.ctx.check(_lib.ebmg_query_level(self.h, level, C.byref(n), C.byref(n2)), "ebmg_query_level")
        return n.value, n2.value

    def level_arrays(self, level):
        """(tag, primary, sec_cell) host arrays of a multigrid level."""
        n, n2 = self.level_size(level)
        tag = np.zeros(n, np.uint8)
        prim = np.zeros(n, np.int8)
        sc = np.zeros(max(1, n2), np.int64)
        self.ctx.check(_lib.ebmg_export_level(self.h, level, _ptr(tag), _ptr(prim), _ptr(sc)), "ebmg_export_level")
        return tag, prim, sc[:n2]

    def operator(self, level=0):
        """Host CSR (scipy) of the level's operator over its N + N2 unknowns."""
        import scipy.sparse as sp
        n, n2 = self.level_size(level)
        nd = n + n2
        nnz = C.c_int64()
        self.ctx.check(_lib.ebmg_export_operator(self.h, level, C.byref(nnz), None, None, None), "export")
        rp = np.zeros(nd + 1, np.int64)
        cols = np.zeros(nnz.value, np.int64)
        vals = np.zeros(nnz.value)
        self.ctx.check(_lib.ebmg_export_operator(self.h, level, C.byref(nnz), _ptr(rp), _ptr(cols), _ptr(vals)),
                       "export")
        return sp.csr_matrix((vals, cols, rp), shape=(nd, nd))

    def rhs(self, rho=None, sigma=None, bc_values=None, obj_values=None):
        rho = _host_f64(self.prob.rho if rho is None else rho).ravel()
        sig = self.prob.sigma if sigma is None else sigma
        sig = None if sig is None else _host_f64(sig).ravel()
        bcv = _host_f64(bc_values)
        ov = _host_f64(obj_values)
        b = np.zeros(self.N + self.N2)
        self.ctx.check(_lib.ebmg_export_rhs(self.h, _ptr(rho), _ptr(sig), _ptr(bcv), _ptr(ov), _ptr(b)),
                       "ebmg_export_rhs")
        return b

    # -- device calls (torch tensors) -------------------------------------------
    def solve(self, rho, phi, sigma=None, phi2=None, E=None, rtol=1e-10, max_cycles=100, bc_values=None,
              obj_values=None, check=True):
        info = SolveInfo()
        bcv = _host_f64(bc_values)
        ov = _host_f64(obj_values)
        args = self._solve_args(rho, phi, sigma, phi2, E)
        st = _lib.ebmg_solve(self.h, args[0], args[1], _ptr(bcv), _ptr(ov), float(rtol), int(max_cycles),
                             *args[2:], C.byref(info))
        if check:
            self.ctx.check(st, "ebmg_solve")
        return st, info.as_dict()

    def submit(self, rho, phi, sigma=None, phi2=None, E=None, rtol=1e-10, max_cycles=100, bc_values=None,
               obj_values=None):
        """Queue the solve on the context's worker; returns its ticket (collect
        it with ``ctx.poll`` / ``ctx.wait``). The tensors are kept referenced
        until then."""
        bcv = _host_f64(bc_values)
        ov = _host_f64(obj_values)
        t = C.c_uint64()
        args = self._solve_args(rho, phi, sigma, phi2, E)
        self.ctx.check(_lib.ebmg_submit(self.h, args[0], args[1], _ptr(bcv), _ptr(ov), float(rtol),
                                        int(max_cycles), *args[2:], C.byref(t)),
                       "ebmg_submit")
        self.ctx._held[t.value] = (rho, sigma, phi, phi2, E)
        return t.value

    def _solve_args(self, rho, phi, sigma, phi2, E):
        c, N, N2 = self.ctx, self.N, self.N2
        return (_dev(c, rho, N, "rho"), _dev(c, sigma, N, "sigma", True), _dev(c, phi, N, "phi"),
                _dev(c, phi2, N2, "phi2", True), _dev(c, E, self.prob.dim * N, "E", True))

    def apply(self, phi, phi2, out, out2):
        c, N, N2 = self.ctx, self.N, self.N2
        self.ctx.check(_lib.ebmg_apply(self.h, _dev(c, phi, N, "phi"), _dev(c, phi2, N2, "phi2", N2 == 0),
                                       _dev(c, out, N, "out"), _dev(c, out2, N2, "out2", N2 == 0)), "ebmg_apply")

    def apply_noalloc(self, phi, phi2, out, out2):
        """As ``apply``, through the entry point that allocates nothing; the
        result is queued on the context's stream (not waited for)."""
        c, N, N2 = self.ctx, self.N, self.N2
        self.ctx.check(_lib.ebmg_apply_noalloc(self.h, _dev(c, phi, N, "phi"), _dev(c, phi2, N2, "phi2", N2 == 0),
                                               _dev(c, out, N, "out"), _dev(c, out2, N2, "out2", N2 == 0)),
                       "ebmg_apply_noalloc")

    def efield(self, phi, phi2, E, sigma=None, bc_values=None, obj_values=None):
        c, N, N2 = self.ctx, self.N, self.N2
        bcv = _host_f64(bc_values)
        ov = _host_f64(obj_values)
        self.ctx.check(_lib.ebmg_efield(self.h, _dev(c, phi, N, "phi"), _dev(c, phi2, N2, "phi2", True),
                                        _dev(c, sigma, N, "sigma", True), _ptr(bcv), _ptr(ov),
                                        _dev(c, E, self.prob.dim * N, "E")), "ebmg_efield")

    def advect(self, n_in, u, dt, n_out, inflow=None):
        """One advection step of a density on the gas phase: n_in, n_out
        device tensors of N cells, u a list of dim device face-velocity
        tensors (faces normal to d: the d extent plus one)."""
        c, N, dim = self.ctx, self.N, self.prob.dim
        if len(u) != dim:
            raise EbmgError(ERR_ARG, f"{dim} face velocity arrays expected")
        nfd = []
        for d in range(dim):
            m = 1
            for e in range(dim):
                m *= self.prob.n[e] + (1 if e == d else 0)
            nfd.append(_dev(c, u[d], m, f"u[{d}]"))
        iv = _host_f64(inflow)
        self.ctx.check(_lib.ebmg_advect(self.h, _dev(c, n_in, N, "n_in"), nfd[0], nfd[1], nfd[2] if dim == 3 else None,
                                        float(dt), _ptr(iv), _dev(c, n_out, N, "n_out")), "ebmg_advect")

    def tuning(self, level):
        """(smoother variant: 0 split, 1 tile, 2 + c z-march in tile ZM_TILES[c],
        OOP_VARIANT one-launch colour phases; split sweep ms; chosen or best
        fused sweep ms) from the setup autotuner; level -1: (first tail level
        or -1, V-cycle ms without tail, V-cycle ms chosen)."""
        f, a, b = C.c_int32(), C.c_double(), C.c_double()
        self.ctx.check(_lib.ebmg_query_tuning(self.h, level, C.byref(f), C.byref(a), C.byref(b)), "tuning")
        return f.value, a.value, b.value

    def smooth(self, level, variant, sweeps, x, b):
        """Template-cell red/black sweeps on level ``level`` (device FP64 x, b)."""
        n = sum(self.level_size(level))
        self.ctx.check(_lib.ebmg_smooth(self.h, level, variant, sweeps, _dev(self.ctx, x, n, "x"),
                                        _dev(self.ctx, b, n, "b")), "ebmg_smooth")

    def restrict_residual(self, level, form, x, b, bc):
        """The V-cycle's residual of level ``level`` restricted into the next
        level's right-hand side ``bc`` (device FP64 tensors; form 0 the
        solver's kernels, 1 the fused pair kernel, 2 separate kernels)."""
        n = sum(self.level_size(level))
        nc = sum(self.level_size(level + 1))
        self.ctx.check(_lib.ebmg_restrict_residual(self.h, level, form, _dev(self.ctx, x, n, "x"),
                                                   _dev(self.ctx, b, n, "b"), _dev(self.ctx, bc, nc, "bc")),
                       "ebmg_restrict_residual")

    def time_kernel(self, which, level=0, reps=50):
        """(mean ms per launch, algorithmic bytes per launch) of a kernel."""
        ms, by = C.c_double(), C.c_double()
        self.ctx.check(_lib.ebmg_time_kernel(self.h, which, level, reps, C.byref(ms), C.byref(by)),
                       "ebmg_time_kernel")
        return ms.value, by.value

    def kernel_timing(self, which, level, enable):
        """Start (enable=True) or stop in-solve event timing of the level's
        sweep launches (which=0) or FP64 residual launches (which=1);
        stopping returns (launches, mean ms, algorithmic bytes per launch)."""
        n, ms, by = C.c_int64(), C.c_double(), C.c_double()
        self.ctx.check(_lib.ebmg_kernel_timing(self.h, int(which), int(level), 1 if enable else 0, C.byref(n),
                                               C.byref(ms), C.byref(by)), "ebmg_kernel_timing")
        return n.value, ms.value, by.value

    def set_coefficients(self, prob):
        """Take the coefficients and boundary data of ``prob`` (same grid, no
        embedded objects) without a new setup."""
        o = Options()
        C.memmove(C.byref(o), C.byref(self.options), C.sizeof(Options))
        o.alpha, o.beta, o.a_gas, o.a_diel, o.b_gas = prob.alpha, prob.beta, prob.a_gas, prob.a_diel, prob.b_gas
        _, _, bc, _ = _c_problem(prob)
        self.ctx.check(_lib.ebmg_set_coefficients(self.h, C.byref(o), C.byref(bc)), "ebmg_set_coefficients")
        self.options = o
        self.prob = prob

    def release(self):
        if getattr(self, "h", None):
            _lib.ebmg_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


# z-marching smoother tiles (x, y, planes, wide fetch), in the library's configuration order;
# the configurations in ZM_QUAD run the quad form (four cells of a row per
# thread), with the occupancy bound of their launch
ZM_TILES = [(64, 8, 32, False), (64, 16, 32, False), (32, 16, 32, False), (64, 8, 16, False), (128, 8, 32, False),
            (32, 8, 32, False), (32, 32, 32, False), (64, 16, 32, True), (128, 8, 32, True), (32, 32, 32, True),
            (64, 16, 8, False), (64, 16, 32, False), (128, 16, 32, False), (128, 8, 32, False)]
ZM_QUAD = {11: 2, 12: 2, 13: 2}


def zm_kernel(t, c, zin=False):
    """Kernel name of z-marching configuration c for element type t."""
    tx, ty, kz, wide = ZM_TILES[c]
    if c in ZM_QUAD:
        return f"k_rb_zq3<{t},{tx},{ty},{kz},{ZM_QUAD[c]},{str(zin).lower()}>"
    return f"k_rb_zm3<{t},{tx},{ty},{kz},{str(wide).lower()},{str(zin).lower()}>"
OOP_VARIANT = 2 + len(ZM_TILES)      # tuning code of the one-launch colour phases
SMOOTH_OOP = 3 + len(ZM_TILES)       # ebmg_smooth variant of the one-launch colour phases
SMOOTH_OOP_ROWS = 4 + len(ZM_TILES)  # the same with each phase's explicit rows relaxed
SMOOTH_FUSED_ROWS = 5 + len(ZM_TILES)  # fused sweeps, each followed by the explicit rows' Jacobi passes

BATCH_LEVELSYNC = 2    # every phase one launch over all boxes (default)
BATCH_PERSISTENT = 1   # one persistent launch, one workgroup per box


class Batch:
    """Independent boxes (one dimension, one precision) solved together,
    level-synchronously (``batch=BATCH_LEVELSYNC``, the default) or by one
    persistent launch (``batch=BATCH_PERSISTENT``); each box keeps the
    boundary values given here."""

    def __init__(self, ctx, probs, **opts):
        self.ctx = ctx
        self.probs = list(probs)
        nb = len(self.probs)
        boxes = (Box * nb)()
        bcs = (DomainBC * nb)()
        optv = (Options * nb)()
        nobj = (C.c_int32 * nb)()
        objp = (_vp * nb)()
        keep = []
        for i, pr in enumerate(self.probs):
            box, objs, bc, sdf = _c_problem(pr)
            boxes[i] = box
            bcs[i] = bc
            optv[i] = make_options(pr, **opts)
            nobj[i] = len(pr.objects)
            objp[i] = C.cast(objs, _vp)
            keep.append((objs, sdf))
        h = _vp()
        st = _lib.ebmg_setup_batch(ctx.h, nb, boxes, nobj, objp, bcs, optv, C.byref(h))
        keep = None
        ctx.check(st, "ebmg_setup_batch")
        self.h = h
        n, n2, by = C.c_int64(), C.c_int64(), C.c_int64()
        ctx.check(_lib.ebmg_query_batch(h, C.byref(n), C.byref(n2), C.byref(by)), "ebmg_query_batch")
        self.cells, self.cells2, self.device_bytes = n.value, n2.value, by.value
        self.sizes = []
        for i in range(nb):
            ni, n2i = C.c_int64(), C.c_int64()
            ctx.check(_lib.ebmg_query_batch_box(h, i, C.byref(ni), C.byref(n2i)), "ebmg_query_batch_box")
            self.sizes.append((ni.value, n2i.value))

    def time_level0(self, which, reps=20):
        """(mean ms, algorithmic bytes) of the finest-level template sweeps
        (which 0) or explicit-row Jacobi passes (1) over every box."""
        ms, by = C.c_double(), C.c_double()
        self.ctx.check(_lib.ebmg_time_batch_kernel(self.h, int(which), int(reps), C.byref(ms), C.byref(by)),
                       "ebmg_time_batch_kernel")
        return ms.value, by.value

    def tuning(self):
        """Setup choices: dict(mode, tail_cells, wide_levels, candidates=[(cells, V-cycle ms)])."""
        mode, tc, wl, nc = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        cc = (C.c_int32 * 8)()
        ms = (C.c_double * 8)()
        self.ctx.check(_lib.ebmg_query_batch_tuning(self.h, C.byref(mode), C.byref(tc), C.byref(wl), C.byref(nc),
                                                    cc, ms), "ebmg_query_batch_tuning")
        return dict(mode=mode.value, tail_cells=tc.value, wide_levels=wl.value,
                    candidates=[(cc[k], ms[k]) for k in range(nc.value)])

    def solve(self, rho, phi, sigma=None, phi2=None, rtol=1e-10, max_cycles=100, check=True):
        """rho, phi (and optionally sigma, phi2) are lists of device tensors,
        one per box (entries of sigma / phi2 may be None)."""
        nb = len(self.probs)
        c = self.ctx

        def arr(xs, name, which, nullable):
            if xs is None:
                return None
            if len(xs) != nb:
                raise EbmgError(ERR_ARG, f"{name}: {len(xs)} tensors for {nb} boxes")
            return (_vp * nb)(*[_dev(c, x, self.sizes[i][which], f"{name}[{i}]", nullable or self.sizes[i][which] == 0)
                               for i, x in enumerate(xs)])
        if rho is None or phi is None:
            raise EbmgError(ERR_ARG, "rho and phi are required")
        infos = (SolveInfo * nb)()
        st = _lib.ebmg_solve_batch(self.h, arr(rho, "rho", 0, False), arr(sigma, "sigma", 0, True), float(rtol),
                                   int(max_cycles), arr(phi, "phi", 0, False), arr(phi2, "phi2", 1, False), infos)
        if check:
            self.ctx.check(st, "ebmg_solve_batch")
        return st, [infos[i].as_dict() for i in range(nb)]

    def release(self):
        if getattr(self, "h", None):
            _lib.ebmg_release_batch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Family:
    """Helmholtz operators on one geometry (``workloads.Problem`` members that
    share the grid, the objects and the boundary kinds; coefficients and
    boundary data may differ), set up once with a shared hierarchy
    structure and solved together, each member on its own stream."""

    def __init__(self, ctx, probs, **opts):
        self.ctx = ctx
        self.probs = list(probs)
        nm = len(self.probs)
        box, objs, _, sdf = _c_problem(self.probs[0])
        bcs = (DomainBC * nm)()
        optv = (Options * nm)()
        for k, pr in enumerate(self.probs):
            bcs[k] = _c_bc(pr)
            optv[k] = make_options(pr, **opts)
        h = _vp()
        st = _lib.ebmg_setup_family(ctx.h, C.byref(box), len(self.probs[0].objects), objs, nm, bcs, optv,
                                    C.byref(h))
        sdf = None
        ctx.check(st, "ebmg_setup_family")
        self.h = h
        m, n, n2, by, sh = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        ctx.check(_lib.ebmg_query_family(h, C.byref(m), C.byref(n), C.byref(n2), C.byref(by), C.byref(sh)),
                  "ebmg_query_family")
        self.nmem, self.N, self.N2, self.device_bytes, self.shared_bytes = m.value, n.value, n2.value, by.value, sh.value

    def solve(self, rho, phi, sigma=None, phi2=None, rtol=1e-10, max_cycles=100, check=True):
        """rho, phi (and optionally sigma, phi2): lists of nmem device tensors
        or None (a member whose rho is None is not solved). Returns (status,
        [per-member status], [per-member info])."""
        nm = self.nmem
        c = self.ctx
        if len(rho) != nm or len(phi) != nm:
            raise EbmgError(ERR_ARG, f"{nm} members: rho and phi need {nm} entries")

        def arr(xs, name, n, nullable):
            if xs is None:
                return None
            if len(xs) != nm:
                raise EbmgError(ERR_ARG, f"{name}: {len(xs)} entries for {nm} members")
            return (_vp * nm)(*[None if (rho[k] is None) else _dev(c, x, n, f"{name}[{k}]", nullable)
                                for k, x in enumerate(xs)])
        infos = (SolveInfo * nm)()
        sts = (C.c_int * nm)()
        st = _lib.ebmg_solve_family(self.h, arr(rho, "rho", self.N, True), arr(sigma, "sigma", self.N, True),
                                    float(rtol), int(max_cycles), arr(phi, "phi", self.N, False),
                                    arr(phi2, "phi2", self.N2, self.N2 == 0), infos, sts)
        if check:
            self.ctx.check(st, "ebmg_solve_family")
        return st, [sts[k] for k in range(nm)], [infos[k].as_dict() for k in range(nm)]

    def release(self):
        if getattr(self, "h", None):
            _lib.ebmg_release_family(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Mesh:
    """A closed triangle mesh resident on the device for signed distances
    (vertices (nv, 3), triangles (nt, 3) counter-clockwise seen from outside)."""

    def __init__(self, ctx, verts, tris):
        self.ctx = ctx
        v = np.ascontiguousarray(verts, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
            raise EbmgError(ERR_ARG, "verts (nv, 3) and tris (nt, 3) expected")
        h = _vp()
        ctx.check(_lib.ebmg_mesh_create(ctx.h, len(v), _ptr(v), len(t), _ptr(t), C.byref(h)), "ebmg_mesh_create")
        self.h = h
        nt, nn, dp, by = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64()
        ctx.check(_lib.ebmg_mesh_query(h, C.byref(nt), C.byref(nn), C.byref(dp), C.byref(by)), "ebmg_mesh_query")
        self.ntri, self.nnode, self.depth, self.device_bytes = nt.value, nn.value, dp.value, by.value

    def sdf(self, n, h, lo, out):
        """Signed distance at the nodes of an n[0] x n[1] x n[2]-cell box
        (out: device float64 tensor of prod(n+1) entries); returns the number
        of boxes and triangles the search examined."""
        box = Box()
        box.dim = 3
        for d in range(3):
            box.n[d] = int(n[d])
            box.lo[d] = float(lo[d])
        box.h = float(h)
        m = (int(n[0]) + 1) * (int(n[1]) + 1) * (int(n[2]) + 1)
        vis = C.c_int64()
        self.ctx.check(_lib.ebmg_mesh_sdf(self.h, C.byref(box), _dev(self.ctx, out, m, "out"), C.byref(vis)),
                       "ebmg_mesh_sdf")
        return vis.value

    def release(self):
        if getattr(self, "h", None):
            _lib.ebmg_mesh_release(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass


class Amr:
    """A nested AMR hierarchy set up from a ``workloads.AmrProblem`` (a tree
    of boxes, box 0 the domain): composite solves and applies; per-box lists
    of device tensors in the order of ``amr.levels``."""

    def __init__(self, ctx, amr, **opts):
        self.ctx = ctx
        self.amr = amr
        L = len(amr.levels)
        boxes = (Box * L)()
        keep, objarrs = [], []
        nobj = (C.c_int32 * L)()
        levs = (C.c_int32 * L)(*[int(getattr(lv, "level", l)) for l, lv in enumerate(amr.levels)])
        ptrs = (_vp * L)()
        for l, lv in enumerate(amr.levels):
            box, objs, _, sdf = _c_problem(lv.prob)
            boxes[l] = box
            keep.append(sdf)
            objarrs.append(objs)
            nobj[l] = len(lv.prob.objects)
            ptrs[l] = C.cast(objs, _vp)
        bc = _c_bc(amr.levels[0].prob)
        self.options = make_options(amr.levels[0].prob, **opts)
        h = _vp()
        st = _lib.ebmg_setup_amr(ctx.h, L, boxes, levs, nobj, ptrs, C.byref(bc), C.byref(self.options), C.byref(h))
        del keep, objarrs
        ctx.check(st, "ebmg_setup_amr")
        self.h = h
        self.L = L
        self.N, self.N2, self.covered = [], [], []
        for l in range(L):
            n, n2, nc, by = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
            ctx.check(_lib.ebmg_query_amr(h, l, C.byref(n), C.byref(n2), C.byref(nc), C.byref(by)), "ebmg_query_amr")
            self.N.append(n.value)
            self.N2.append(n2.value)
            self.covered.append(nc.value)
            self.device_bytes = by.value

    def _arrays(self, ts, sizes, name, nullable=False):
        arr = (_vp * self.L)()
        for l in range(self.L):
            t = ts[l] if ts is not None else None
            if sizes[l] == 0 and t is None:
                arr[l] = None
                continue
            arr[l] = _dev(self.ctx, t, sizes[l], f"{name}[{l}]", nullable=nullable and sizes[l] == 0)
        return arr

    def solve(self, rho, phi, phi2=None, rtol=1e-10, max_iters=200, check=True):
        """rho, phi (and phi2 where a level has second-phase unknowns): lists
        of device float64 tensors per level. Returns (status, info dict)."""
        if len(rho) != self.L or len(phi) != self.L:
            raise EbmgError(ERR_ARG, f"{self.L} levels expected")
        r = self._arrays(rho, self.N, "rho")
        x = self._arrays(phi, self.N, "phi")
        x2 = self._arrays(phi2, self.N2, "phi2", nullable=True) if phi2 is not None else None
        if x2 is None and any(self.N2):
            raise EbmgError(ERR_ARG, "phi2 needed for levels with second-phase unknowns")
        info = SolveInfo()
        st = _lib.ebmg_solve_amr(self.h, r, float(rtol), int(max_iters), x, x2, C.byref(info))
        if check:
            self.ctx.check(st, "ebmg_solve_amr")
        return st, info.as_dict()

    def apply(self, phi, out, phi2=None, out2=None):
        x = self._arrays(phi, self.N, "phi")
        y = self._arrays(out, self.N, "out")
        x2 = self._arrays(phi2, self.N2, "phi2", nullable=True) if phi2 is not None else None
        y2 = self._arrays(out2, self.N2, "out2", nullable=True) if out2 is not None else None
        self.ctx.check(_lib.ebmg_apply_amr(self.h, x, x2, y, y2), "ebmg_apply_amr")

    def release(self):
        if self.h:
            _lib.ebmg_release_amr(self.h)
            self.h = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
