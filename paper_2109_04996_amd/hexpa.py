"""ctypes binding of libhexpa.so: the ``hx_*`` C entry points under the same names.

Argument marshalling only. Every step of the operator and the solves runs in
the HIP library; this module converts torch tensors to device pointers and
torch streams to ``hipStream_t`` handles, and turns negative status codes into
``HexpaError``. It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HEXPA_LIB") or os.path.join(_PKG, "libhexpa.so")

HX_OK, HX_EINVAL, HX_ERANGE, HX_EUNSUPPORTED, HX_EGEOM, HX_ENOCONV, HX_EBREAKDOWN, HX_EHIP, HX_ENOMEM = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
HX_GAUSS, HX_GLL = 0, 1
HX_MASS, HX_DIFFUSION, HX_HELMHOLTZ, HX_LOR = 0, 1, 2, 3
HX_FP64, HX_FP32, HX_BF16, HX_BF16_SPLIT = 0, 1, 2, 3
HX_PC_NONE, HX_PC_JACOBI, HX_PC_CHEBYSHEV, HX_PC_MLP, HX_PC_PMG = 0, 1, 2, 3, 4
HX_SOLVE_FP64, HX_SOLVE_IR, HX_SOLVE_MIXED = 0, 1, 2
HX_SCATTER_COLORS, HX_SCATTER_GATHER = 0, 1

STATUS_NAMES = {0: "HX_OK", -1: "HX_EINVAL", -2: "HX_ERANGE", -3: "HX_EUNSUPPORTED", -4: "HX_EGEOM",
                -5: "HX_ENOCONV", -6: "HX_EBREAKDOWN", -7: "HX_EHIP", -8: "HX_ENOMEM"}


class HexpaError(RuntimeError):
    def __init__(self, code: int, func: str, msg: str):
        super().__init__(f"{func} -> {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class hx_mesh_stats(C.Structure):
    _fields_ = [("p", C.c_int), ("ncolors", C.c_int), ("nelem", C.c_int64), ("nnodes", C.c_int64),
                ("nfree", C.c_int64), ("nuntouched", C.c_int64), ("max_color", C.c_int64),
                ("nstrips", C.c_int64), ("nstrip_colors", C.c_int64), ("nstrip_groups", C.c_int64),
                ("index_mode", C.c_int)]


class hx_kappa_rff(C.Structure):
    _fields_ = [("M", C.c_int), ("omega", C.POINTER(C.c_double)), ("phase", C.POINTER(C.c_double)),
                ("scale", C.c_double), ("shift", C.c_double)]


class hx_op_stats(C.Structure):
    _fields_ = [("p", C.c_int), ("q", C.c_int), ("qrule", C.c_int), ("kind", C.c_int), ("ncomp", C.c_int),
                ("nnodes", C.c_int64), ("nelem", C.c_int64), ("qdata_bytes", C.c_int64),
                ("index_bytes", C.c_int64)]


class hx_solve_opts(C.Structure):
    _fields_ = [("mode", C.c_int), ("precond", C.c_int), ("rtol", C.c_double), ("maxit", C.c_int),
                ("check_every", C.c_int), ("use_x0", C.c_int), ("cheb_degree", C.c_int),
                ("cheb_ratio", C.c_double), ("cheb_prec", C.c_int), ("lanczos_steps", C.c_int),
                ("inner_rtol", C.c_double), ("inner_maxit", C.c_int), ("inner_qdata", C.c_int),
                ("flexible", C.c_int), ("mlp", C.c_void_p), ("fallback", C.c_int), ("stall_window", C.c_int),
                ("stall_factor", C.c_double), ("mlp_mode", C.c_int), ("graph", C.c_int), ("pmg", C.c_void_p),
                ("scatter", C.c_int), ("reliable_delta", C.c_double)]


class hx_pmg_opts(C.Structure):
    _fields_ = [("smooth_degree", C.c_int), ("smooth_ratio", C.c_double), ("lanczos_steps", C.c_int),
                ("coarse_maxit", C.c_int), ("coarse_rtol", C.c_double), ("prec", C.c_int),
                ("smoother_mlp", C.c_void_p), ("cycles", C.c_int)]


class hx_train_opts(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64)]


class hx_train_info(C.Structure):
    _fields_ = [("steps", C.c_int64), ("first_loss", C.c_double), ("final_loss", C.c_double),
                ("seconds", C.c_double)]


class hx_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int), ("outer_iterations", C.c_int), ("operator_applies", C.c_int),
                ("rel_residual", C.c_double), ("true_rel_residual", C.c_double), ("lam_max", C.c_double),
                ("setup_seconds", C.c_double), ("solve_seconds", C.c_double), ("fallback_used", C.c_int),
                ("fallback_iterations", C.c_int), ("fallback_reason", C.c_int)]


_VP, _I64, _I32P = C.c_void_p, C.c_int64, C.c_void_p

# (name, restype, argtypes): every symbol include/hexpa.h declares
SIGNATURES = [
    ("hx_last_error", C.c_char_p, []),
    ("hx_version", C.c_char_p, []),
    ("hx_mesh_nodes_trilinear", C.c_int, [C.c_int, _I64, _VP, _I64, _VP, _VP, _I64, _VP]),
    ("hx_mesh_create", C.c_int, [C.c_int, _I64, _I64, _VP, _VP, _VP, C.POINTER(_VP)]),
    ("hx_mesh_get_stats", C.c_int, [_VP, C.POINTER(hx_mesh_stats)]),
    ("hx_mesh_get_order", C.c_int, [_VP, _VP, _VP]),
    ("hx_mesh_plan", C.c_int, [C.c_int, _I64, _I64, _VP, _VP, _VP, C.POINTER(_VP)]),
    ("hx_mesh_plan_arrays", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("hx_mesh_destroy", None, [_VP]),
    ("hx_basis_create", C.c_int, [C.c_int, C.c_int, C.c_int, C.POINTER(_VP)]),
    ("hx_basis_get_tables", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    ("hx_basis_destroy", None, [_VP]),
    ("hx_op_create", C.c_int, [_VP, _VP, C.c_int, C.c_int, C.POINTER(hx_kappa_rff), _VP, C.POINTER(_VP)]),
    ("hx_op_create_helmholtz", C.c_int, [_VP, _VP, C.c_int, C.c_double, C.c_double, C.POINTER(hx_kappa_rff), _VP,
                                         C.POINTER(_VP)]),
    ("hx_op_create_lor", C.c_int, [_VP, C.POINTER(hx_kappa_rff), _VP, C.POINTER(_VP)]),
    ("hx_op_lor_matrix", C.c_int, [_VP, C.POINTER(C.c_int), _VP, _VP]),
    ("hx_op_apply", C.c_int, [_VP, _VP, _VP, _VP]),
    ("hx_op_apply_f32", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("hx_op_apply_bf16", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("hx_op_apply_elem", C.c_int, [_VP, _VP, _VP, _VP]),
    ("hx_op_diagonal", C.c_int, [_VP, _VP, _VP]),
    ("hx_op_get_stats", C.c_int, [_VP, C.POINTER(hx_op_stats)]),
    ("hx_op_destroy", None, [_VP]),
    ("hx_solve_opts_default", None, [C.POINTER(hx_solve_opts)]),
    ("hx_mlp_create", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_uint64, C.POINTER(_VP)]),
    ("hx_mlp_get_shape", C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("hx_mlp_set_params", C.c_int, [_VP, _VP]),
    ("hx_mlp_get_params", C.c_int, [_VP, _VP]),
    ("hx_mlp_forward", C.c_int, [_VP, C.c_int, _VP, _I64, _VP, _VP]),
    ("hx_mlp_loss_grad", C.c_int, [_VP, _VP, _VP, _I64, C.POINTER(C.c_double), _VP, _VP]),
    ("hx_train_opts_default", None, [C.c_void_p]),
    ("hx_mlp_train", C.c_int, [_VP, _VP, _VP, _I64, _VP, _VP, _VP]),
    ("hx_mlp_save", C.c_int, [_VP, C.c_char_p]),
    ("hx_mlp_load", C.c_int, [C.c_char_p, C.POINTER(_VP)]),
    ("hx_mlp_destroy", None, [_VP]),
    ("hx_op_mlp_features", C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("hx_op_mlp_targets", C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("hx_op_mlp_precond", C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP]),
    ("hx_pcg_solve", C.c_int, [_VP, _VP, _VP, C.POINTER(hx_solve_opts), C.POINTER(hx_solve_info), _VP]),
    ("hx_pcg_solve_noalloc", C.c_int, [_VP, _VP, _VP, C.POINTER(hx_solve_opts), C.POINTER(hx_solve_info), _VP]),
    ("hx_pmg_opts_default", None, [C.POINTER(hx_pmg_opts)]),
    ("hx_pmg_create", C.c_int, [_VP, C.c_int, C.POINTER(hx_pmg_opts), _VP, C.POINTER(_VP)]),
    ("hx_pmg_levels", C.c_int, [_VP]),
    ("hx_pmg_lambda_max", C.c_int, [_VP, C.c_int, C.POINTER(C.c_double)]),
    ("hx_pmg_vcycle", C.c_int, [_VP, _VP, _VP, _VP]),
    ("hx_pmg_prolong", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("hx_pmg_restrict", C.c_int, [_VP, C.c_int, _VP, _VP, _VP]),
    ("hx_pmg_destroy", None, [_VP]),
]

_lib = None


def load(path: str = LIB_PATH):
    """Load libhexpa.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2109_04996_amd.build` "
                          "(the operator has no CPU fallback)")
    # PyTorch first: its HIP runtime must be the one in the process, or a library loaded ahead of it
    # leaves torch seeing no GPU (the buffers and streams passed here are torch's)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    for name, res, args in SIGNATURES:
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(code: int, func: str):
    if code != HX_OK:
        raise HexpaError(code, func, load().hx_last_error().decode())


def _ptr(t) -> int:
    """Device or host pointer of a torch tensor or numpy array (contiguous)."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        if not t.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be C-contiguous")
        return t.ctypes.data
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


# ---------------------------------------------------------------------------- thin wrappers, same names

def hx_version() -> str:
    return load().hx_version().decode()


def hx_last_error() -> str:
    return load().hx_last_error().decode()


def hx_mesh_nodes_trilinear(p, elem_verts: np.ndarray, verts: np.ndarray, elem_nodes: np.ndarray, nnodes: int):
    ev = np.ascontiguousarray(elem_verts, dtype=np.int64)
    vv = np.ascontiguousarray(verts, dtype=np.float64)
    en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
    out = np.zeros((nnodes, 3))
    _check(load().hx_mesh_nodes_trilinear(p, ev.shape[0], _ptr(ev), vv.shape[0], _ptr(vv), _ptr(en), nnodes,
                                          _ptr(out)), "hx_mesh_nodes_trilinear")
    return out


def hx_mesh_create(p, elem_nodes: np.ndarray, node_xyz: np.ndarray, dirichlet: np.ndarray | None):
    en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
    xyz = np.ascontiguousarray(node_xyz, dtype=np.float64)
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    h = C.c_void_p()
    _check(load().hx_mesh_create(p, en.shape[0], xyz.shape[0], _ptr(en), _ptr(xyz), _ptr(d), C.byref(h)),
           "hx_mesh_create")
    return h


def hx_mesh_plan(p, elem_nodes: np.ndarray, node_xyz: np.ndarray, dirichlet: np.ndarray | None):
    en = np.ascontiguousarray(elem_nodes, dtype=np.int32)
    xyz = np.ascontiguousarray(node_xyz, dtype=np.float64)
    d = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    h = C.c_void_p()
    _check(load().hx_mesh_plan(p, en.shape[0], xyz.shape[0], _ptr(en), _ptr(xyz), _ptr(d), C.byref(h)),
           "hx_mesh_plan")
    return h


def hx_mesh_plan_arrays(plan, p: int) -> dict:
    st = hx_mesh_get_stats(plan)
    P = p + 1
    E, G = st["nelem"], st["nstrip_groups"]
    out = dict(idx=np.zeros((E, P ** 3), np.int32), own=np.zeros((E, P * P), np.uint16),
               strip_elems=np.zeros((G, 8), np.int32), strip_link=np.zeros(G, np.uint8),
               strip_own=np.zeros((E, P * P), np.uint16),
               strip_color_start=np.zeros(st["nstrip_colors"] + 1, np.int64))
    strips = st["nstrips"] > 0
    _check(load().hx_mesh_plan_arrays(plan, _ptr(out["idx"]), _ptr(out["own"]),
                                      _ptr(out["strip_elems"]) if strips else None,
                                      _ptr(out["strip_link"]) if strips else None,
                                      _ptr(out["strip_own"]) if strips else None,
                                      _ptr(out["strip_color_start"]) if strips else None), "hx_mesh_plan_arrays")
    return out


def hx_mesh_get_stats(mesh) -> dict:
    s = hx_mesh_stats()
    _check(load().hx_mesh_get_stats(mesh, C.byref(s)), "hx_mesh_get_stats")
    return {k: getattr(s, k) for k, _ in s._fields_}


def hx_mesh_get_order(mesh, nelem: int, ncolors: int):
    order = np.zeros(nelem, np.int32)
    cs = np.zeros(ncolors + 1, np.int64)
    _check(load().hx_mesh_get_order(mesh, _ptr(order), _ptr(cs)), "hx_mesh_get_order")
    return order, cs


def hx_mesh_destroy(mesh):
    load().hx_mesh_destroy(mesh)


def hx_basis_create(p, q, qrule):
    h = C.c_void_p()
    _check(load().hx_basis_create(p, q, qrule, C.byref(h)), "hx_basis_create")
    return h


def hx_basis_get_tables(basis, p, q):
    P = p + 1
    nodes, qp, qw = np.zeros(P), np.zeros(q), np.zeros(q)
    interp, grad = np.zeros((q, P)), np.zeros((q, P))
    _check(load().hx_basis_get_tables(basis, _ptr(nodes), _ptr(qp), _ptr(qw), _ptr(interp), _ptr(grad)),
           "hx_basis_get_tables")
    return dict(nodes=nodes, qpts=qp, qweights=qw, interp=interp, grad=grad)


def hx_basis_destroy(basis):
    load().hx_basis_destroy(basis)


def _kappa_struct(kappa: dict | None):
    """(hx_kappa_rff or None, arrays to keep alive during the call)."""
    if kappa is None:
        return None, None
    om = np.ascontiguousarray(kappa["omega"], dtype=np.float64)
    ph = np.ascontiguousarray(kappa["phase"], dtype=np.float64)
    kp = hx_kappa_rff(om.shape[0], om.ctypes.data_as(C.POINTER(C.c_double)),
                      ph.ctypes.data_as(C.POINTER(C.c_double)), float(kappa["scale"]), float(kappa["shift"]))
    return kp, (om, ph)


def hx_op_create(mesh, basis, kind, ncomp, kappa: dict | None = None, stream=None):
    h = C.c_void_p()
    kp, keep = _kappa_struct(kappa)
    _check(load().hx_op_create(mesh, basis, kind, ncomp, C.byref(kp) if kp is not None else None, _stream(stream),
                               C.byref(h)), "hx_op_create")
    del keep
    return h


def hx_op_create_helmholtz(mesh, basis, ncomp, alpha, beta, kappa: dict | None = None, stream=None):
    h = C.c_void_p()
    kp, keep = _kappa_struct(kappa)
    _check(load().hx_op_create_helmholtz(mesh, basis, ncomp, float(alpha), float(beta),
                                         C.byref(kp) if kp is not None else None, _stream(stream), C.byref(h)),
           "hx_op_create_helmholtz")
    del keep
    return h


def hx_op_create_lor(mesh, kappa: dict | None = None, stream=None):
    h = C.c_void_p()
    kp, keep = _kappa_struct(kappa)
    _check(load().hx_op_create_lor(mesh, C.byref(kp) if kp is not None else None, _stream(stream), C.byref(h)),
           "hx_op_create_lor")
    del keep
    return h


def hx_op_lor_matrix(op, nnodes: int):
    """(W, cols [W][nnodes] int32, vals [W][nnodes] float64) of a low-order refined operator."""
    w = C.c_int()
    _check(load().hx_op_lor_matrix(op, C.byref(w), None, None), "hx_op_lor_matrix")
    cols = np.empty((w.value, nnodes), dtype=np.int32)
    vals = np.empty((w.value, nnodes), dtype=np.float64)
    _check(load().hx_op_lor_matrix(op, C.byref(w), cols.ctypes.data_as(C.c_void_p), vals.ctypes.data_as(C.c_void_p)),
           "hx_op_lor_matrix")
    return w.value, cols, vals


def hx_op_apply(op, x, y, stream=None):
    _check(load().hx_op_apply(op, _ptr(x), _ptr(y), _stream(stream)), "hx_op_apply")


def hx_op_apply_f32(op, qdata_prec, x, y, stream=None):
    _check(load().hx_op_apply_f32(op, qdata_prec, _ptr(x), _ptr(y), _stream(stream)), "hx_op_apply_f32")


def hx_op_apply_bf16(op, x, y, stream=None, prec=HX_BF16):
    _check(load().hx_op_apply_bf16(op, prec, _ptr(x), _ptr(y), _stream(stream)), "hx_op_apply_bf16")


def hx_op_apply_elem(op, x, y_e, stream=None):
    _check(load().hx_op_apply_elem(op, _ptr(x), _ptr(y_e), _stream(stream)), "hx_op_apply_elem")


def hx_op_diagonal(op, diag, stream=None):
    _check(load().hx_op_diagonal(op, _ptr(diag), _stream(stream)), "hx_op_diagonal")


def hx_op_get_stats(op) -> dict:
    s = hx_op_stats()
    _check(load().hx_op_get_stats(op, C.byref(s)), "hx_op_get_stats")
    return {k: getattr(s, k) for k, _ in s._fields_}


def hx_op_destroy(op):
    load().hx_op_destroy(op)


def hx_solve_opts_default(**overrides) -> hx_solve_opts:
    o = hx_solve_opts()
    load().hx_solve_opts_default(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def _solve(name, op, b, x, opts: hx_solve_opts, stream, raise_on_error):
    info = hx_solve_info()
    code = getattr(load(), name)(op, _ptr(b), _ptr(x), C.byref(opts), C.byref(info), _stream(stream))
    d = {k: getattr(info, k) for k, _ in info._fields_}
    d["status"] = STATUS_NAMES.get(code, code)
    if raise_on_error and code != HX_OK:
        raise HexpaError(code, name, hx_last_error())
    return d


def hx_pcg_solve(op, b, x, opts: hx_solve_opts, stream=None, raise_on_error=True):
    return _solve("hx_pcg_solve", op, b, x, opts, stream, raise_on_error)


HX_NOALLOC_MAX_DOFS = 1048576


def hx_pcg_solve_noalloc(op, b, x, opts: hx_solve_opts, stream=None, raise_on_error=True):
    return _solve("hx_pcg_solve_noalloc", op, b, x, opts, stream, raise_on_error)


# ---------------------------------------------------------------------------- p-multigrid

def hx_pmg_opts_default(**overrides) -> hx_pmg_opts:
    o = hx_pmg_opts()
    load().hx_pmg_opts_default(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def hx_pmg_create(ops, opts: hx_pmg_opts, stream=None):
    arr = (C.c_void_p * len(ops))(*[o.value if isinstance(o, C.c_void_p) else o for o in ops])
    h = C.c_void_p()
    _check(load().hx_pmg_create(arr, len(ops), C.byref(opts), _stream(stream), C.byref(h)), "hx_pmg_create")
    return h


def hx_pmg_levels(mg) -> int:
    return load().hx_pmg_levels(mg)


def hx_pmg_lambda_max(mg, level) -> float:
    v = C.c_double()
    _check(load().hx_pmg_lambda_max(mg, level, C.byref(v)), "hx_pmg_lambda_max")
    return v.value


def hx_pmg_vcycle(mg, r, z, stream=None):
    _check(load().hx_pmg_vcycle(mg, _ptr(r), _ptr(z), _stream(stream)), "hx_pmg_vcycle")


def hx_pmg_prolong(mg, level, x_coarse, y_fine, stream=None):
    _check(load().hx_pmg_prolong(mg, level, _ptr(x_coarse), _ptr(y_fine), _stream(stream)), "hx_pmg_prolong")


def hx_pmg_restrict(mg, level, r_fine, y_coarse, stream=None):
    _check(load().hx_pmg_restrict(mg, level, _ptr(r_fine), _ptr(y_coarse), _stream(stream)), "hx_pmg_restrict")


def hx_pmg_destroy(mg):
    load().hx_pmg_destroy(mg)


# ---------------------------------------------------------------------------- network

def hx_mlp_create(n_in, n_hidden, n_out, seed=7):
    h = C.c_void_p()
    _check(load().hx_mlp_create(n_in, n_hidden, n_out, seed, C.byref(h)), "hx_mlp_create")
    return h


def hx_mlp_get_shape(net):
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    _check(load().hx_mlp_get_shape(net, C.byref(a), C.byref(b), C.byref(c)), "hx_mlp_get_shape")
    return a.value, b.value, c.value


def mlp_param_count(n_in, n_hidden, n_out):
    return n_hidden * (n_in + 1) + n_out * (n_hidden + 1)


def hx_mlp_set_params(net, params: np.ndarray):
    a = np.ascontiguousarray(params, dtype=np.float32)
    _check(load().hx_mlp_set_params(net, _ptr(a)), "hx_mlp_set_params")


def hx_mlp_get_params(net) -> np.ndarray:
    out = np.zeros(mlp_param_count(*hx_mlp_get_shape(net)), np.float32)
    _check(load().hx_mlp_get_params(net, _ptr(out)), "hx_mlp_get_params")
    return out


def hx_mlp_forward(net, prec, X, Y, stream=None):
    _check(load().hx_mlp_forward(net, prec, _ptr(X), X.shape[0], _ptr(Y), _stream(stream)), "hx_mlp_forward")


def hx_mlp_loss_grad(net, X, T, stream=None):
    loss = C.c_double()
    g = np.zeros(mlp_param_count(*hx_mlp_get_shape(net)), np.float32)
    _check(load().hx_mlp_loss_grad(net, _ptr(X), _ptr(T), X.shape[0], C.byref(loss), _ptr(g), _stream(stream)),
           "hx_mlp_loss_grad")
    return loss.value, g


def hx_train_opts_default(**overrides) -> hx_train_opts:
    o = hx_train_opts()
    load().hx_train_opts_default(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def hx_mlp_train(net, X, T, opts: hx_train_opts, stream=None) -> dict:
    info = hx_train_info()
    _check(load().hx_mlp_train(net, _ptr(X), _ptr(T), X.shape[0], C.byref(opts), C.byref(info), _stream(stream)),
           "hx_mlp_train")
    return {k: getattr(info, k) for k, _ in info._fields_}


def hx_mlp_save(net, path: str):
    _check(load().hx_mlp_save(net, path.encode()), "hx_mlp_save")


def hx_mlp_load(path: str):
    h = C.c_void_p()
    _check(load().hx_mlp_load(path.encode(), C.byref(h)), "hx_mlp_load")
    return h


def hx_mlp_destroy(net):
    load().hx_mlp_destroy(net)


def hx_op_mlp_features(op, r, X, rnorm, stream=None):
    _check(load().hx_op_mlp_features(op, _ptr(r), _ptr(X), _ptr(rnorm), _stream(stream)), "hx_op_mlp_features")


def hx_op_mlp_targets(op, err, rnorm, T, stream=None):
    _check(load().hx_op_mlp_targets(op, _ptr(err), _ptr(rnorm), _ptr(T), _stream(stream)), "hx_op_mlp_targets")


def hx_op_mlp_precond(op, net, r, z, mode=0, stream=None):
    _check(load().hx_op_mlp_precond(op, net, mode, _ptr(r), _ptr(z), _stream(stream)), "hx_op_mlp_precond")
