"""ctypes binding of libfc (include/fc.h).

Argument marshalling only: every computation runs in the native library.
Device buffers are passed as raw pointers; the helpers accept torch tensors
(FP64, on the GPU) and take their data_ptr(), and streams default to
torch's current stream.  Loading fails loudly when libfc.so is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfc.so")

FC_OK, FC_E_ARG, FC_E_NOMEM, FC_E_DEVICE, FC_E_NOTCONV, FC_E_BREAKDOWN, \
    FC_E_NAN, FC_E_UNSUPPORTED = range(8)
STATUS_NAMES = {0: "OK", 1: "E_ARG", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_NOTCONV",
                5: "E_BREAKDOWN", 6: "E_NAN", 7: "E_UNSUPPORTED"}
PDE = {"poisson": 0, "elasticity": 1}
DOMAIN = {"voids": 0, "inclusions": 1}
STORE_F64, STORE_F32, STORE_BF16 = 1, 2, 4
STOP = {"precond": 0, "residual": 1}
MODE = {"f64": 0, "ir_f32": 1, "ir_bf16": 2, "s_f32": 3, "s_bf16": 4, "learned": 5}
BLOCK_KIND = {"element": 0, "vertex_patch": 1}

# every symbol include/fc.h declares
EXPORTS = [
    "fc_setup", "fc_assemble", "fc_host_system_info", "fc_host_system_export",
    "fc_setup_from_host", "fc_host_system_destroy", "fc_setup_from_matrix",
    "fc_problem_info", "fc_get_rhs", "fc_get_eta", "fc_export", "fc_apply_A",
    "fc_precond_build", "fc_precond_info", "fc_get_block_inverse", "fc_apply_M",
    "fc_pcg_solve", "fc_problem_destroy", "fc_precond_destroy", "fc_last_error",
    "fc_batch_create", "fc_batch_info", "fc_pcg_solve_batch", "fc_batch_destroy",
    "fc_model_param_count", "fc_model_create", "fc_model_get_params", "fc_model_set_params",
    "fc_model_forward", "fc_model_loss_grad", "fc_model_train", "fc_model_destroy",
    "fc_learned_attach", "fc_coarse_grid", "fc_coarse_channels", "fc_coarse_restrict",
    "fc_coarse_prolong", "fc_coarse_apply", "fc_learned_stats", "fc_learned_snapshots",
    "fc_learned_validate", "fc_precond_lowprec_info", "fc_spmv_info",
    "fc_precond_block_dropped", "fc_pcg_solve_noalloc", "fc_precond_shape",
]


class FcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libfc {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class ProblemDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n", C.c_int32), ("p", C.c_int32), ("pde", C.c_int32),
                ("alpha", C.c_double), ("quad_depth", C.c_int32), ("domain", C.c_int32),
                ("n_shapes", C.c_int32), ("shape_centre", C.POINTER(C.c_double)),
                ("shape_semi", C.POINTER(C.c_double)), ("n_modes", C.c_int32),
                ("mode_k", C.POINTER(C.c_double)), ("mode_amp", C.POINTER(C.c_double)),
                ("mode_phase", C.POINTER(C.c_double)), ("E", C.c_double), ("nu", C.c_double),
                ("traction", C.c_double * 3), ("clamp_zmin", C.c_int32),
                ("discard_fictitious", C.c_int32)]


class PrecondOpts(C.Structure):
    _fields_ = [("eta_bar", C.c_double), ("eps", C.c_double), ("stabilize", C.c_int32),
                ("store_mask", C.c_uint32), ("block_kind", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int64), ("stop", C.c_int32),
                ("mode", C.c_int32), ("check_every", C.c_int32), ("inner_tol", C.c_double),
                ("history_dev", C.c_void_p), ("timing", C.c_int32), ("fcg_m", C.c_int32)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int64), ("outer_iters", C.c_int64),
                ("rel_res_true", C.c_double), ("rel_res_prec", C.c_double),
                ("status", C.c_int32), ("ms_solve", C.c_double), ("ms_spmv", C.c_double),
                ("ms_schwarz", C.c_double), ("n_timed", C.c_int64), ("fallbacks", C.c_int64)]


_lib = None


def load():
    """Load libfc.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FcError(FC_E_UNSUPPORTED,
                      f"{LIB_PATH} is missing; build it with "
                      "`python -m paper_1809_00828_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.c_void_p
    P = C.POINTER
    sig = {
        "fc_setup": [P(ProblemDesc), vp, P(vp)],
        "fc_assemble": [P(ProblemDesc), P(vp)],
        "fc_host_system_info": [vp, P(i64), P(i64), P(i64), P(i32), P(i32)],
        "fc_host_system_export": [vp, vp, vp, vp, vp, vp, vp],
        "fc_setup_from_host": [vp, vp, P(vp)],
        "fc_setup_from_matrix": [i64, i32, vp, vp, vp, vp, i64, i32, vp, vp, vp, P(vp)],
        "fc_problem_info": [vp, P(i64), P(i64), P(i64), P(i32), P(i32)],
        "fc_get_rhs": [vp, dp, vp],
        "fc_get_eta": [vp, vp],
        "fc_export": [vp, vp, vp, vp, vp],
        "fc_apply_A": [vp, dp, dp, vp],
        "fc_precond_build": [vp, P(PrecondOpts), vp, P(vp)],
        "fc_precond_info": [vp, P(i64), P(i64), P(i64), P(i64)],
        "fc_precond_lowprec_info": [vp, P(i64), P(i64)],
        "fc_spmv_info": [vp, P(i32), P(i32)],
        "fc_get_block_inverse": [vp, i64, vp],
        "fc_precond_block_dropped": [vp, vp],
        "fc_precond_shape": [vp, P(i32), P(i32)],
        "fc_apply_M": [vp, dp, dp, vp],
        "fc_pcg_solve": [vp, vp, dp, dp, P(SolveOpts), P(SolveInfo), vp],
        "fc_pcg_solve_noalloc": [vp, vp, dp, dp, P(SolveOpts), P(SolveInfo), vp],
        "fc_batch_create": [i32, vp, vp, i32, vp, P(vp)],
        "fc_batch_info": [vp, P(i64), P(i32), P(i32), C.c_char_p, i64],
        "fc_pcg_solve_batch": [vp, vp, vp, P(SolveOpts), vp, vp],
        "fc_model_param_count": [vp, i32, P(i64)],
        "fc_model_create": [vp, i32, vp, P(vp)],
        "fc_model_get_params": [vp, vp],
        "fc_model_set_params": [vp, vp],
        "fc_model_forward": [vp, i32, i32, dp, dp, vp],
        "fc_model_loss_grad": [vp, i32, i32, dp, dp, P(C.c_double), vp, vp],
        "fc_model_train": [vp, i64, i32, dp, dp, P(TrainOpts), vp, vp],
        "fc_learned_attach": [vp, vp],
        "fc_coarse_grid": [vp, P(i32)],
        "fc_coarse_channels": [vp, dp, dp],
        "fc_coarse_restrict": [vp, dp, dp, vp],
        "fc_coarse_prolong": [vp, dp, C.c_double, dp, vp],
        "fc_coarse_apply": [vp, dp, dp, P(C.c_double), vp],
        "fc_learned_stats": [vp, P(i64), P(i64)],
        "fc_learned_snapshots": [vp, dp, dp, i32, vp, i32, C.c_double, dp, dp, P(i32), vp],
        "fc_learned_validate": [vp, dp, C.c_double, i32, P(i32), P(SolveInfo), P(SolveInfo), vp],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    for name in ("fc_problem_destroy", "fc_precond_destroy", "fc_host_system_destroy",
                 "fc_batch_destroy", "fc_model_destroy"):
        f = getattr(lib, name)
        f.argtypes = [vp]
        f.restype = None
    lib.fc_last_error.argtypes = []
    lib.fc_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(status):
    if status != FC_OK:
        msg = load().fc_last_error().decode(errors="replace")
        raise FcError(status, msg)


def _dptr(t):
    """Device pointer of a torch tensor (FP64 contiguous), or an int."""
    if isinstance(t, int):
        return t
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise FcError(FC_E_ARG, "expected a contiguous FP64 CUDA tensor")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def make_desc(d: dict):
    """ctypes description of a problem dict (see fcgen); returns (desc, keep)
    where keep holds the arrays the pointers refer to."""
    dim = d["dim"]
    centre = np.ascontiguousarray([s["centre"] for s in d["shapes"]], dtype=np.float64).ravel()
    semi = np.ascontiguousarray([s["semi"] for s in d["shapes"]], dtype=np.float64).ravel()
    mk = np.ascontiguousarray([m["k"] for m in d["modes"]], dtype=np.float64).ravel()
    ma = np.ascontiguousarray([m["amp"] for m in d["modes"]], dtype=np.float64)
    mp = np.ascontiguousarray([m["phase"] for m in d["modes"]], dtype=np.float64)
    keep = [centre, semi, mk, ma, mp]
    dp = C.POINTER(C.c_double)
    desc = ProblemDesc()
    desc.dim, desc.n, desc.p = dim, d["n"], d["p"]
    desc.pde = PDE[d["pde"]]
    desc.alpha = d["alpha"]
    desc.quad_depth = d["quad_depth"]
    desc.domain = DOMAIN[d["domain"]]
    desc.n_shapes = len(d["shapes"])
    desc.shape_centre = centre.ctypes.data_as(dp)
    desc.shape_semi = semi.ctypes.data_as(dp)
    desc.n_modes = len(d["modes"])
    desc.mode_k = mk.ctypes.data_as(dp)
    desc.mode_amp = ma.ctypes.data_as(dp)
    desc.mode_phase = mp.ctypes.data_as(dp)
    desc.E, desc.nu = d["E"], d["nu"]
    t = list(d["traction"]) + [0.0] * (3 - len(d["traction"]))
    desc.traction = (C.c_double * 3)(*t[:3])
    desc.clamp_zmin = 1 if d.get("clamp_zmin") else 0
    desc.discard_fictitious = 1 if d.get("discard_fictitious") else 0
    return desc, keep


class HostSystem:
    """Host-assembled system (fc_assemble); needs no GPU."""

    def __init__(self, desc: dict):
        lib = load()
        cd, self._keep = make_desc(desc)
        h = C.c_void_p()
        _check(lib.fc_assemble(C.byref(cd), C.byref(h)))
        self._h = h

    def info(self):
        lib = load()
        n, nnzb, nel = C.c_int64(), C.c_int64(), C.c_int64()
        m, bd = C.c_int32(), C.c_int32()
        _check(lib.fc_host_system_info(self._h, C.byref(n), C.byref(nnzb), C.byref(nel),
                                       C.byref(m), C.byref(bd)))
        return {"n_dofs": n.value, "nnzb": nnzb.value, "n_el": nel.value, "m": m.value,
                "bsr_dim": bd.value}

    def export(self):
        inf = self.info()
        bd = inf["bsr_dim"]
        rp = np.zeros(inf["n_dofs"] // bd + 1, np.int32)
        col = np.zeros(inf["nnzb"], np.int32)
        val = np.zeros(inf["nnzb"] * bd * bd, np.float64)
        rhs = np.zeros(inf["n_dofs"], np.float64)
        ed = np.zeros(inf["n_el"] * inf["m"], np.int32)
        eta = np.zeros(inf["n_el"], np.float64)
        _check(load().fc_host_system_export(self._h, _np_ptr(rp), _np_ptr(col), _np_ptr(val),
                                            _np_ptr(rhs), _np_ptr(ed), _np_ptr(eta)))
        return {"rowptr": rp, "col": col, "val": val.reshape(-1, bd, bd), "rhs": rhs,
                "elem_dofs": ed.reshape(inf["n_el"], inf["m"]), "eta": eta, **inf}

    def upload(self, stream=None):
        h = C.c_void_p()
        _check(load().fc_setup_from_host(self._h, C.c_void_p(_stream(stream)), C.byref(h)))
        return Problem(h)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fc_host_system_destroy(self._h)
            self._h = None


class Problem:
    def __init__(self, handle):
        self._h = handle
        self._info = None

    @classmethod
    def setup(cls, desc: dict, stream=None):
        cd, keep = make_desc(desc)
        h = C.c_void_p()
        _check(load().fc_setup(C.byref(cd), C.c_void_p(_stream(stream)), C.byref(h)))
        return cls(h)

    @classmethod
    def from_matrix(cls, n, bsr_dim, rowptr, col, val, rhs, elem_dofs, eta, stream=None):
        rowptr = np.ascontiguousarray(rowptr, np.int32)
        col = np.ascontiguousarray(col, np.int32)
        val = np.ascontiguousarray(val, np.float64).ravel()
        rhs = np.ascontiguousarray(rhs, np.float64)
        elem_dofs = np.ascontiguousarray(elem_dofs, np.int32)
        eta = np.ascontiguousarray(eta, np.float64)
        h = C.c_void_p()
        _check(load().fc_setup_from_matrix(
            int(n), int(bsr_dim), _np_ptr(rowptr), _np_ptr(col), _np_ptr(val), _np_ptr(rhs),
            int(elem_dofs.shape[0]), int(elem_dofs.shape[1]), _np_ptr(elem_dofs), _np_ptr(eta),
            C.c_void_p(_stream(stream)), C.byref(h)))
        return cls(h)

    def info(self):
        if self._info is None:
            n, nnzb, nel = C.c_int64(), C.c_int64(), C.c_int64()
            m, bd = C.c_int32(), C.c_int32()
            _check(load().fc_problem_info(self._h, C.byref(n), C.byref(nnzb), C.byref(nel),
                                          C.byref(m), C.byref(bd)))
            g, lat = C.c_int32(), C.c_int32()
            _check(load().fc_spmv_info(self._h, C.byref(g), C.byref(lat)))
            self._info = {"n_dofs": n.value, "nnzb": nnzb.value, "n_el": nel.value,
                          "m": m.value, "bsr_dim": bd.value, "spmv_group": g.value,
                          "lattice_columns": lat.value >= 1, "sliced": lat.value == 2}
        return self._info

    @property
    def n(self):
        return self.info()["n_dofs"]

    def rhs(self, out, stream=None):
        _check(load().fc_get_rhs(self._h, C.c_void_p(_dptr(out)), C.c_void_p(_stream(stream))))
        return out

    def eta(self):
        e = np.zeros(self.info()["n_el"], np.float64)
        _check(load().fc_get_eta(self._h, _np_ptr(e)))
        return e

    def export(self):
        inf = self.info()
        bd = inf["bsr_dim"]
        rp = np.zeros(inf["n_dofs"] // bd + 1, np.int32)
        col = np.zeros(inf["nnzb"], np.int32)
        val = np.zeros(inf["nnzb"] * bd * bd, np.float64)
        ed = np.zeros(inf["n_el"] * inf["m"], np.int32)
        _check(load().fc_export(self._h, _np_ptr(rp), _np_ptr(col), _np_ptr(val), _np_ptr(ed)))
        return {"rowptr": rp, "col": col, "val": val.reshape(-1, bd, bd),
                "elem_dofs": ed.reshape(inf["n_el"], inf["m"])}

    def apply_A(self, x, y, stream=None):
        _check(load().fc_apply_A(self._h, C.c_void_p(_dptr(x)), C.c_void_p(_dptr(y)),
                                 C.c_void_p(_stream(stream))))
        return y

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fc_problem_destroy(self._h)
            self._h = None


class Precond:
    def __init__(self, problem: Problem, eta_bar=1.0, eps=1e-13, stabilize=True,
                 store=STORE_F64, block_kind="element", stream=None):
        o = PrecondOpts(float(eta_bar), float(eps), 1 if stabilize else 0, int(store),
                        BLOCK_KIND[block_kind])
        h = C.c_void_p()
        _check(load().fc_precond_build(problem._h, C.byref(o), C.c_void_p(_stream(stream)),
                                       C.byref(h)))
        self._h = h
        self.problem = problem     # keeps the problem alive as long as this
        self.block_kind = block_kind
        m, kind = C.c_int32(), C.c_int32()
        _check(load().fc_precond_shape(h, C.byref(m), C.byref(kind)))
        self.m = m.value

    def info(self):
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(load().fc_precond_info(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        e, f = C.c_int64(), C.c_int64()
        _check(load().fc_precond_lowprec_info(self._h, C.byref(e), C.byref(f)))
        return {"n_blocks": a.value, "n_fallback": b.value, "n_eig_blocks": c.value,
                "n_dropped": d.value, "n_f32_blocks": e.value, "n_f32_from_f64": f.value}

    def block_dropped(self):
        """Eigenvalues dropped by the threshold in every block."""
        out = np.zeros(self.info()["n_blocks"], np.int32)
        _check(load().fc_precond_block_dropped(self._h, _np_ptr(out)))
        return out

    def block_inverse(self, k):
        out = np.zeros((self.m, self.m), np.float64)
        _check(load().fc_get_block_inverse(self._h, int(k), _np_ptr(out)))
        return out

    def apply_M(self, r, z, stream=None):
        _check(load().fc_apply_M(self._h, C.c_void_p(_dptr(r)), C.c_void_p(_dptr(z)),
                                 C.c_void_p(_stream(stream))))
        return z

    # ---- learned coarse correction (fc_learned_* / fc_coarse_*)
    def attach(self, model):
        """Attach a Model for mode="learned" (None detaches)."""
        _check(load().fc_learned_attach(self._h, model._h if model is not None else None))
        self._model = model        # the library keeps a reference

    def coarse_grid(self):
        g = C.c_int32()
        _check(load().fc_coarse_grid(self._h, C.byref(g)))
        return g.value

    def coarse_channels(self, eta, mask):
        _check(load().fc_coarse_channels(self._h, C.c_void_p(_fptr(eta)),
                                         C.c_void_p(_fptr(mask))))

    def coarse_restrict(self, r, rc, stream=None):
        _check(load().fc_coarse_restrict(self._h, C.c_void_p(_dptr(r)), C.c_void_p(_dptr(rc)),
                                          C.c_void_p(_stream(stream))))
        return rc

    def coarse_prolong(self, y, gamma, z, stream=None):
        _check(load().fc_coarse_prolong(self._h, C.c_void_p(_fptr(y)), float(gamma),
                                         C.c_void_p(_dptr(z)), C.c_void_p(_stream(stream))))
        return z

    def coarse_apply(self, y, v, stream=None):
        g = C.c_double()
        _check(load().fc_coarse_apply(self._h, C.c_void_p(_fptr(y)), C.c_void_p(_dptr(v)),
                                       C.byref(g), C.c_void_p(_stream(stream))))
        return g.value

    def validate(self, b, tol=1e-8, fcg_m=1, stream=None):
        """fc_learned_validate: returns (use_network, plain info, learned info)."""
        use = C.c_int32()
        ip, il = SolveInfo(), SolveInfo()
        _check(load().fc_learned_validate(self._h, C.c_void_p(_dptr(b)), float(tol),
                                          int(fcg_m), C.byref(use), C.byref(ip), C.byref(il),
                                          C.c_void_p(_stream(stream))))
        return bool(use.value), _info_dict(ip), _info_dict(il)

    def learned_stats(self):
        a, d = C.c_int64(), C.c_int64()
        _check(load().fc_learned_stats(self._h, C.byref(a), C.byref(d)))
        return {"applied": a.value, "dropped": d.value}

    def snapshots(self, b, x_star, iters, xin, t, kind="e-Sr", tol=1e-8, stream=None):
        """Training pairs at the listed iterations (fc_learned_snapshots);
        returns how many were written."""
        it = np.ascontiguousarray(iters, dtype=np.int32)
        k = C.c_int32()
        _check(load().fc_learned_snapshots(
            self._h, C.c_void_p(_dptr(b)), C.c_void_p(_dptr(x_star)), int(it.size), _np_ptr(it),
            {"e-Sr": 0, "e": 1, "coarse": 2}[kind], float(tol), C.c_void_p(_fptr(xin)), C.c_void_p(_fptr(t)),
            C.byref(k), C.c_void_p(_stream(stream))))
        return k.value

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fc_precond_destroy(self._h)
            self._h = None


def pcg_solve(problem: Problem, precond: Precond, b, x, tol=1e-10, maxit=300000,
              stop="precond", mode="f64", check_every=16, inner_tol=1e-4, history=None,
              timing=False, stream=None, raise_on_error=False, fcg_m=1):
    """Run fc_pcg_solve; returns the info dict (status included)."""
    o = SolveOpts(float(tol), int(maxit), STOP[stop], MODE[mode], int(check_every),
                  float(inner_tol), C.c_void_p(_dptr(history)) if history is not None else None,
                  int(timing), int(fcg_m))
    info = SolveInfo()
    st = load().fc_pcg_solve(problem._h, precond._h, C.c_void_p(_dptr(b)), C.c_void_p(_dptr(x)),
                             C.byref(o), C.byref(info), C.c_void_p(_stream(stream)))
    if st not in (FC_OK, FC_E_NOTCONV, FC_E_BREAKDOWN, FC_E_NAN) or (raise_on_error and st):
        _check(st)
    return _info_dict(info, st)


def pcg_solve_noalloc(problem: Problem, precond: Precond, b, x, tol=1e-10, maxit=300000,
                      stop="precond", check_every=16, history=None, stream=None,
                      raise_on_error=False):
    """Run fc_pcg_solve_noalloc (FP64 PCG with the library's static device
    scratch instead of an allocated workspace); returns the info dict."""
    o = SolveOpts(float(tol), int(maxit), STOP[stop], MODE["f64"], int(check_every), 1e-4,
                  C.c_void_p(_dptr(history)) if history is not None else None, 0, 1)
    info = SolveInfo()
    st = load().fc_pcg_solve_noalloc(problem._h, precond._h, C.c_void_p(_dptr(b)),
                                     C.c_void_p(_dptr(x)), C.byref(o), C.byref(info),
                                     C.c_void_p(_stream(stream)))
    if st not in (FC_OK, FC_E_NOTCONV, FC_E_BREAKDOWN, FC_E_NAN) or (raise_on_error and st):
        _check(st)
    return _info_dict(info, st)


def _info_dict(info, st=FC_OK):
    return {"iters": info.iters, "outer_iters": info.outer_iters,
            "rel_res_true": info.rel_res_true, "rel_res_prec": info.rel_res_prec,
            "status": STATUS_NAMES.get(info.status if st == FC_OK else st, st),
            "ms_solve": info.ms_solve, "ms_spmv": info.ms_spmv,
            "ms_schwarz": info.ms_schwarz, "n_timed": info.n_timed,
            "fallbacks": info.fallbacks}


class Batch:
    """Many problems solved together (fc_batch_create / fc_pcg_solve_batch)."""

    def __init__(self, problems, preconds, autotune=True, stream=None):
        if len(problems) != len(preconds) or not problems:
            raise FcError(FC_E_ARG, "need one preconditioner per problem")
        self.problems = list(problems)
        self.preconds = list(preconds)
        k = len(problems)
        hp = (C.c_void_p * k)(*[p._h.value for p in problems])
        hc = (C.c_void_p * k)(*[c._h.value for c in preconds])
        h = C.c_void_p()
        _check(load().fc_batch_create(k, hp, hc, 1 if autotune else 0,
                                      C.c_void_p(_stream(stream)), C.byref(h)))
        self._h = h

    def info(self):
        tot, a, b = C.c_int64(), C.c_int32(), C.c_int32()
        buf = C.create_string_buffer(1 << 16)
        _check(load().fc_batch_info(self._h, C.byref(tot), C.byref(a), C.byref(b), buf,
                                    len(buf)))
        return {"total_dofs": tot.value, "spmv_classes": a.value, "schwarz_classes": b.value,
                "report": buf.value.decode()}

    def solve(self, bs, xs, tol=1e-8, maxit=300000, stop="precond", check_every=16,
              stream=None):
        k = len(self.problems)
        bp = (C.c_void_p * k)(*[_dptr(t) for t in bs])
        xp = (C.c_void_p * k)(*[_dptr(t) for t in xs])
        o = SolveOpts(float(tol), int(maxit), STOP[stop], 0, int(check_every), 1e-4, None, 0)
        infos = (SolveInfo * k)()
        st = load().fc_pcg_solve_batch(self._h, bp, xp, C.byref(o), infos,
                                       C.c_void_p(_stream(stream)))
        if st not in (FC_OK, FC_E_NOTCONV, FC_E_BREAKDOWN, FC_E_NAN):
            _check(st)
        return [{"iters": i.iters, "status": STATUS_NAMES.get(i.status, i.status),
                 "rel_res_prec": i.rel_res_prec, "rel_res": i.rel_res_true,
                 "ms_solve": i.ms_solve} for i in infos]

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fc_batch_destroy(self._h)
            self._h = None


def _fptr(t):
    """Device pointer of a contiguous FP32 CUDA tensor."""
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise FcError(FC_E_ARG, "expected a contiguous FP32 CUDA tensor")
    return t.data_ptr()


class Model:
    """The learned coarse-correction network (fc_model_*)."""

    def __init__(self, params, ch=(8, 16, 32, 32), in_ch=2):
        self.ch = tuple(int(c) for c in ch)
        self.in_ch = int(in_ch)
        arr = (C.c_int32 * 4)(*self.ch)
        n = C.c_int64()
        _check(load().fc_model_param_count(arr, self.in_ch, C.byref(n)))
        self.n_params = n.value
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.n_params:
            raise FcError(FC_E_ARG, f"expected {self.n_params} parameters, got {p.size}")
        h = C.c_void_p()
        _check(load().fc_model_create(arr, self.in_ch, _np_ptr(p), C.byref(h)))
        self._h = h

    def params(self):
        out = np.zeros(self.n_params, np.float32)
        _check(load().fc_model_get_params(self._h, _np_ptr(out)))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(load().fc_model_set_params(self._h, _np_ptr(p)))

    def forward(self, x, y, stream=None):
        B, _, g = x.shape[0], x.shape[1], x.shape[2]
        _check(load().fc_model_forward(self._h, B, g, C.c_void_p(_fptr(x)),
                                       C.c_void_p(_fptr(y)), C.c_void_p(_stream(stream))))
        return y

    def loss_grad(self, x, t, stream=None):
        B, g = x.shape[0], x.shape[2]
        loss = C.c_double()
        grad = np.zeros(self.n_params, np.float32)
        _check(load().fc_model_loss_grad(self._h, B, g, C.c_void_p(_fptr(x)),
                                         C.c_void_p(_fptr(t)), C.byref(loss), _np_ptr(grad),
                                         C.c_void_p(_stream(stream))))
        return loss.value, grad

    def train(self, x, t, epochs=10, batch=8, lr=1e-3, stream=None):
        n, g = x.shape[0], x.shape[2]
        hist = np.zeros(epochs, np.float64)
        o = TrainOpts(int(epochs), int(batch), float(lr))
        _check(load().fc_model_train(self._h, n, g, C.c_void_p(_fptr(x)), C.c_void_p(_fptr(t)),
                                     C.byref(o), _np_ptr(hist), C.c_void_p(_stream(stream))))
        return hist

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.fc_model_destroy(self._h)
            self._h = None
