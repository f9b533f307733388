"""ctypes binding of ``libyasps.so`` (C ABI in ``include/yasps.h``).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory and the stream.  Loading fails loudly
when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libyasps.so")

OK, E_ARG, E_HIP, E_DOMAIN, E_NONFINITE, E_NOCONV, E_BREAKDOWN, E_UNIMPL, E_LINESEARCH = 0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS_NAMES = {OK: "OK", E_ARG: "E_ARG", E_HIP: "E_HIP", E_DOMAIN: "E_DOMAIN", E_NONFINITE: "E_NONFINITE",
                E_NOCONV: "E_NOCONV", E_BREAKDOWN: "E_BREAKDOWN", E_UNIMPL: "E_UNIMPL",
                E_LINESEARCH: "E_LINESEARCH"}
PT, EE, PE, PP = 0, 1, 2, 3
FP64, MIXED = 0, 1
F_SPACE, X_SPACE = 0, 1
PROJECTED, EXACT = 0, 1
SQLOG, IPC_CLASSIC = 0, 1
INDEX_DEVICE, INDEX_HOST = 0, 1  # yasps_params.index_build

EXPORTS = ["yasps_create", "yasps_set_contacts", "yasps_eval_stencils", "yasps_assemble_bsr", "yasps_pcg",
           "yasps_pcg_noalloc", "yasps_newton_step", "yasps_get_pattern", "yasps_theta_adjoint", "yasps_profile_enable",
           "yasps_profile_query", "yasps_spmv", "yasps_lm_shift", "yasps_set_body_contacts", "yasps_set_surface",
           "yasps_detect", "yasps_get_detected", "yasps_ccd", "yasps_frame", "yasps_destroy", "yasps_last_error"]
K_INERTIA, K_SNH, K_CONTACT, K_ASSEMBLE, K_BLOCKINV, K_SPMV, K_PCG_UPDATE, K_LINESEARCH, K_CLOTH = range(9)
KERNEL_CLASSES = ["inertia", "snh_eval", "contact_eval", "assemble", "block_inverse", "pcg_spmv", "pcg_update",
                  "linesearch", "cloth_eval"]


class Problem(C.Structure):
    _fields_ = [("n_free", C.c_int32), ("n_fixed", C.c_int32), ("x_fixed", C.c_void_p), ("mass", C.c_void_p),
                ("x_tilde", C.c_void_p), ("n_tets", C.c_int32), ("tet_idx", C.c_void_p), ("dm_inv", C.c_void_p),
                ("vol", C.c_void_p), ("mu_lambda", C.c_void_p), ("mu", C.c_double), ("lambda_", C.c_double),
                ("h", C.c_double), ("kappa", C.c_double), ("dhat", C.c_double), ("gravity", C.c_double * 3),
                ("is_static", C.c_int32), ("n_tris", C.c_int32), ("tri_idx", C.c_void_p),
                ("tri_dm_inv", C.c_void_p), ("tri_area", C.c_void_p), ("mu_c", C.c_double), ("lambda_c", C.c_double),
                ("thickness", C.c_double), ("n_hinges", C.c_int32), ("hinge_idx", C.c_void_p),
                ("hinge_rest", C.c_void_p), ("n_bodies", C.c_int32), ("body_mass", C.c_void_p),
                ("body_k", C.c_void_p), ("n_body_verts", C.c_int32), ("body_of", C.c_void_p),
                ("body_rest", C.c_void_p)]


class Contacts(C.Structure):
    _fields_ = [("n_contacts", C.c_int32), ("type", C.c_void_p), ("idx", C.c_void_p), ("ee_eps", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("proj", C.c_int32), ("barrier", C.c_int32), ("index_build", C.c_int32)]


class EvalInfo(C.Structure):
    _fields_ = [("energy", C.c_double), ("e_inertia", C.c_double), ("e_elastic", C.c_double),
                ("e_contact", C.c_double), ("min_d", C.c_double), ("n_active", C.c_int32)]


class BsrView(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("nnzb_static", C.c_int32), ("nnzb_dynamic", C.c_int32),
                ("row_ptr_s", C.c_void_p), ("col_idx_s", C.c_void_p), ("values_s", C.c_void_p),
                ("row_ptr_d", C.c_void_p), ("col_idx_d", C.c_void_p), ("values_d", C.c_void_p),
                ("values_are_f32", C.c_int32), ("grad", C.c_void_p), ("block_inv", C.c_void_p),
                ("nnzb_body", C.c_int32), ("row_ptr_b", C.c_void_p), ("col_idx_b", C.c_void_p),
                ("values_b", C.c_void_p)]


class Surface(C.Structure):
    _fields_ = [("n_points", C.c_int32), ("points", C.c_void_p), ("n_edges", C.c_int32), ("edges", C.c_void_p),
                ("n_tris", C.c_int32), ("tris", C.c_void_p), ("edge_rest_len2", C.c_void_p), ("cell", C.c_double)]


class FrameParams(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_newton", C.c_int32), ("rtol", C.c_double), ("max_iter", C.c_int32),
                ("armijo", C.c_double), ("max_halvings", C.c_int32), ("ccd_s", C.c_double)]


class FrameInfo(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("cg_iters", C.c_int32), ("ls_trials", C.c_int32),
                ("n_contacts_max", C.c_int32), ("e_begin", C.c_double), ("e_end", C.c_double),
                ("alpha_min", C.c_double), ("converged", C.c_int32), ("ms_detect", C.c_float),
                ("ms_newton", C.c_float), ("ms_ccd", C.c_float), ("ms_linesearch", C.c_float)]


class PcgInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("rel_residual", C.c_double), ("status", C.c_int32)]


class NewtonParams(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("max_halvings", C.c_int32), ("armijo", C.c_double),
                ("tie_rtol", C.c_double), ("hessian", C.c_int32), ("shift", C.c_double)]


class NewtonInfo(C.Structure):
    _fields_ = [("e0", C.c_double), ("e1", C.c_double), ("alpha", C.c_double), ("alpha0", C.c_double),
                ("grad_dot_p", C.c_double), ("grad_max", C.c_double), ("step_max", C.c_double), ("cg_iters", C.c_int32), ("cg_rel_residual", C.c_double),
                ("cg_status", C.c_int32), ("ls_trials", C.c_int32), ("ms_eval", C.c_float),
                ("ms_assemble", C.c_float), ("ms_pcg", C.c_float), ("ms_linesearch", C.c_float)]


_lib = None
_hip = None


def lib():
    """Loads libyasps.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2605_23088_amd.build`")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.yasps_create.argtypes = [C.POINTER(P), P, C.POINTER(Problem), C.POINTER(Params)]
        L.yasps_set_contacts.argtypes = [P, C.POINTER(Contacts)]
        L.yasps_set_body_contacts.argtypes = [P, C.POINTER(Contacts)]
        L.yasps_eval_stencils.argtypes = [P, P, C.c_int32, C.POINTER(EvalInfo)]
        L.yasps_assemble_bsr.argtypes = [P, C.POINTER(BsrView)]
        L.yasps_pcg.argtypes = [P, P, P, C.c_double, C.c_int32, C.POINTER(PcgInfo)]
        L.yasps_pcg_noalloc.argtypes = [P, P, P, C.c_double, C.c_int32, C.POINTER(PcgInfo)]
        L.yasps_newton_step.argtypes = [P, P, C.POINTER(NewtonParams), C.POINTER(NewtonInfo)]
        L.yasps_get_pattern.argtypes = [P, C.c_int32, P, P, P]
        L.yasps_theta_adjoint.argtypes = [P, P, P, P, P]
        L.yasps_profile_enable.argtypes = [P, C.c_int32]
        L.yasps_profile_query.argtypes = [P, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_double)]
        L.yasps_spmv.argtypes = [P, P, P]
        L.yasps_lm_shift.argtypes = [P, C.c_double, C.POINTER(C.c_double)]
        L.yasps_set_surface.argtypes = [P, C.POINTER(Surface)]
        L.yasps_detect.argtypes = [P, P, C.POINTER(C.c_int32)]
        L.yasps_get_detected.argtypes = [P, P, P, P]
        L.yasps_ccd.argtypes = [P, P, P, C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.yasps_frame.argtypes = [P, P, P, C.POINTER(FrameParams), C.POINTER(FrameInfo)]
        L.yasps_destroy.argtypes = [P]
        L.yasps_destroy.restype = None
        L.yasps_last_error.argtypes = [P]
        L.yasps_last_error.restype = C.c_char_p
        for f in EXPORTS[:-2]:
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _hiprt():
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so.7")  # the runtime torch already loaded
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    return _hip


class YaspsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


class Yasps:
    """One context of the library bound to a synthetic problem dict (see
    :mod:`paper_2605_23088_amd.synth`).  Problem arrays are uploaded once and
    kept alive here; positions are (n, 3) float64 CUDA tensors over the rows of
    degrees of freedom: the free vertices, then a_1, a_2, a_3, t of each affine
    body (n = n_free + 4 n_bodies)."""

    def __init__(self, prob, device="cuda", precision=FP64, proj=F_SPACE, barrier=SQLOG, contacts=True,
                 index_build=INDEX_DEVICE):
        if not torch.cuda.is_available():
            raise RuntimeError("the yasps library needs a ROCm GPU")
        self.dev = torch.device(device)
        torch.cuda.init()
        L = lib()
        d = self.dev
        f64 = dict(dtype=torch.float64, device=d)
        self.nv = int(prob["n_free"])
        self.nb = int(prob.get("n_bodies", 0))
        self.n = self.nv + 4 * self.nb
        nt = int(prob["tet_idx"].shape[0])
        self.nt = nt
        self._x_fixed = torch.as_tensor(np.asarray(prob["x_fixed"]).reshape(-1, 3), **f64).contiguous()
        self._mass = torch.as_tensor(prob["mass"], **f64).contiguous()
        xt = np.asarray(prob["x_tilde"], np.float64).reshape(-1, 3)
        if self.nb:
            xt = np.concatenate([xt, np.asarray(prob["body_qt"], np.float64).reshape(-1, 3)])
        self._x_tilde = torch.as_tensor(xt, **f64).contiguous()
        self._tet = torch.as_tensor(np.ascontiguousarray(np.asarray(prob["tet_idx"], np.int32).T),
                                    device=d).contiguous()
        self._dm = torch.as_tensor(np.ascontiguousarray(np.asarray(prob["dm_inv"]).reshape(nt, 9).T), **f64)
        self._vol = torch.as_tensor(prob["vol"], **f64).contiguous()
        self._ml = None
        if "mu_t" in prob:
            self._ml = torch.as_tensor(np.stack([prob["mu_t"], prob["lam_t"]]), **f64).contiguous()
        P = Problem()
        P.n_free = self.nv
        P.n_fixed = int(self._x_fixed.shape[0])
        P.x_fixed = _ptr(self._x_fixed)
        P.mass = _ptr(self._mass)
        P.x_tilde = _ptr(self._x_tilde)
        P.n_tets = nt
        P.tet_idx = _ptr(self._tet)
        P.dm_inv = _ptr(self._dm)
        P.vol = _ptr(self._vol)
        P.mu_lambda = _ptr(self._ml)
        P.mu = float(prob.get("mu", 0.0))
        P.lambda_ = float(prob.get("lam", 0.0))
        P.h = float(prob["h"])
        P.kappa = float(prob["kappa"])
        P.dhat = float(prob["dhat"])
        g = np.asarray(prob.get("gravity", [0, 0, -9.81]), np.float64)
        P.gravity = (C.c_double * 3)(*g)
        P.is_static = int(bool(prob.get("static", False)))
        # cloth: membrane triangles and bending hinges, structure-of-arrays
        self.nf = int(len(prob.get("tri_idx", [])))
        self.nh = int(len(prob.get("hinge_idx", [])))
        i32 = dict(dtype=torch.int32, device=d)
        if self.nf:
            nf = self.nf
            self._tri = torch.as_tensor(np.ascontiguousarray(np.asarray(prob["tri_idx"], np.int32).T), **i32)
            self._tdm = torch.as_tensor(np.ascontiguousarray(np.asarray(prob["tri_dm_inv"]).reshape(nf, 4).T), **f64)
            self._tarea = torch.as_tensor(np.asarray(prob["tri_area"], np.float64), **f64).contiguous()
            P.n_tris = nf
            P.tri_idx = _ptr(self._tri)
            P.tri_dm_inv = _ptr(self._tdm)
            P.tri_area = _ptr(self._tarea)
            P.mu_c = float(prob["mu_c"])
            P.lambda_c = float(prob["lam_c"])
            P.thickness = float(prob["thickness"])
        if self.nh:
            nh = self.nh
            self._hin = torch.as_tensor(np.ascontiguousarray(np.asarray(prob["hinge_idx"], np.int32).T), **i32)
            self._hrest = torch.as_tensor(np.ascontiguousarray(np.asarray(prob["hinge_rest"]).reshape(nh, 2).T),
                                          **f64)
            P.n_hinges = nh
            P.hinge_idx = _ptr(self._hin)
            P.hinge_rest = _ptr(self._hrest)
        # affine bodies: M4 [nb][16], k_b [nb], body of each body vertex, rest positions [nbv][3]
        self.nbc = 0
        if self.nb:
            self._bM4 = torch.as_tensor(np.asarray(prob["body_M4"], np.float64).reshape(self.nb, 16), **f64)
            self._bk = torch.as_tensor(np.asarray(prob["body_k"], np.float64).reshape(self.nb), **f64)
            self._bof = torch.as_tensor(np.asarray(prob["abd_body"], np.int32), **i32).contiguous()
            self._brest = torch.as_tensor(np.asarray(prob["abd_rest"], np.float64).reshape(-1, 3), **f64)
            P.n_bodies = self.nb
            P.body_mass = _ptr(self._bM4)
            P.body_k = _ptr(self._bk)
            P.n_body_verts = int(self._bof.shape[0])
            P.body_of = _ptr(self._bof)
            P.body_rest = _ptr(self._brest.contiguous())
        self.params = Params(precision, proj, barrier, index_build)
        self.stream = torch.cuda.current_stream(d)
        ctx = C.c_void_p()
        rc = L.yasps_create(C.byref(ctx), C.c_void_p(self.stream.cuda_stream), C.byref(P), C.byref(self.params))
        if rc != OK:
            raise YaspsError(rc, L.yasps_last_error(None).decode())
        self.ctx = ctx
        self.nc = 0
        if contacts and len(prob.get("ctype", [])):
            self.set_contacts(prob["ctype"], prob["cidx"], prob.get("ee_eps"))
        if contacts and len(prob.get("bctype", [])):
            self.set_body_contacts(prob["bctype"], prob["bcidx"], prob.get("bee_eps"))

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise YaspsError(rc, lib().yasps_last_error(self.ctx).decode())
        return rc

    def close(self):
        if getattr(self, "ctx", None):
            lib().yasps_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ calls
    def set_contacts(self, ctype, cidx, ee_eps=None):
        """Host arrays: types (n_c), vertex ids (n_c, 4) and optionally the
        edge-edge mollifier thresholds (n_c)."""
        ctype = np.asarray(ctype, np.int32)
        cidx = np.asarray(cidx, np.int32).reshape(-1, 4)
        t = torch.as_tensor(ctype, device=self.dev).contiguous()
        i = torch.as_tensor(np.ascontiguousarray(cidx.T), device=self.dev).contiguous()
        e = None if ee_eps is None else torch.as_tensor(np.asarray(ee_eps, np.float64), device=self.dev)
        self.set_contacts_device(t, i, e)

    def set_contacts_device(self, t, i, eps=None):
        """Device tensors in the library's layout: int32 types [n_c], int32 ids
        [4][n_c], float64 mollifier thresholds [n_c] or None."""
        assert t.dtype == torch.int32 and i.dtype == torch.int32 and i.shape == (4, t.shape[0])
        t, i = t.contiguous(), i.contiguous()  # kept alive through the call
        if eps is not None:
            assert eps.dtype == torch.float64 and eps.shape == t.shape
            eps = eps.contiguous()
        Cs = Contacts(int(t.shape[0]), _ptr(t), _ptr(i), _ptr(eps))
        try:
            self._check(lib().yasps_set_contacts(self.ctx, C.byref(Cs)))
        except YaspsError:
            self.nc = 0  # a rejected set leaves the context without contacts
            raise
        self.nc = int(t.shape[0])

    def set_body_contacts(self, ctype, cidx, ee_eps=None):
        """Host arrays: types (n_s), vertex ids (n_s, 4) and optionally the
        edge-edge mollifier thresholds (n_s) of the stencils touching bodies."""
        ctype = np.asarray(ctype, np.int32)
        cidx = np.asarray(cidx, np.int32).reshape(-1, 4)
        t = torch.as_tensor(ctype, device=self.dev).contiguous()
        i = torch.as_tensor(np.ascontiguousarray(cidx.T), device=self.dev).contiguous()
        e = None if ee_eps is None else torch.as_tensor(np.asarray(ee_eps, np.float64), device=self.dev).contiguous()
        Cs = Contacts(int(t.shape[0]), _ptr(t), _ptr(i), _ptr(e))
        try:
            self._check(lib().yasps_set_body_contacts(self.ctx, C.byref(Cs)))
        except YaspsError:
            self.nbc = 0
            raise
        self.nbc = int(t.shape[0])

    def eval(self, x, exact=False, allow=()):
        info = EvalInfo()
        rc = self._check(lib().yasps_eval_stencils(self.ctx, _ptr(x), EXACT if exact else PROJECTED,
                                                   C.byref(info)), allow)
        out = {k: getattr(info, k) for k, _ in EvalInfo._fields_}
        out["status"] = rc
        return out

    def view(self):
        v = BsrView()
        self._check(lib().yasps_assemble_bsr(self.ctx, C.byref(v)))
        return v

    def assemble(self, copy=True):
        """Assembles and returns copies of the BSR parts, gradient and block
        inverses as CUDA tensors."""
        v = self.view()
        if not copy:
            return v
        n = self.n
        vt = torch.float32 if v.values_are_f32 else torch.float64
        out = dict(
            row_ptr_s=self._dev_copy(v.row_ptr_s, n + 1, torch.int32),
            col_idx_s=self._dev_copy(v.col_idx_s, v.nnzb_static, torch.int32),
            values_s=self._dev_copy(v.values_s, 9 * v.nnzb_static, vt).view(-1, 3, 3),
            grad=self._dev_copy(v.grad, 3 * n, torch.float64).view(n, 3),
            block_inv=self._dev_copy(v.block_inv, 9 * n, torch.float64).view(n, 3, 3),
        )
        if v.nnzb_dynamic:
            out["row_ptr_d"] = self._dev_copy(v.row_ptr_d, n + 1, torch.int32)
            out["col_idx_d"] = self._dev_copy(v.col_idx_d, v.nnzb_dynamic, torch.int32)
            out["values_d"] = self._dev_copy(v.values_d, 9 * v.nnzb_dynamic, vt).view(-1, 3, 3)
        if v.nnzb_body:
            out["row_ptr_b"] = self._dev_copy(v.row_ptr_b, n + 1, torch.int32)
            out["col_idx_b"] = self._dev_copy(v.col_idx_b, v.nnzb_body, torch.int32)
            out["values_b"] = self._dev_copy(v.values_b, 9 * v.nnzb_body, vt).view(-1, 3, 3)
        return out

    def _dev_copy(self, ptr, count, dtype):
        t = torch.empty(count, dtype=dtype, device=self.dev)
        if count:
            rc = _hiprt().hipMemcpyAsync(C.c_void_p(t.data_ptr()), C.c_void_p(ptr), t.numel() * t.element_size(),
                                         3, C.c_void_p(self.stream.cuda_stream))
            if rc != 0:
                raise RuntimeError(f"hipMemcpyAsync failed ({rc})")
        self.stream.synchronize()
        return t

    def pcg(self, b, rtol=1e-8, max_iter=20000, allow=(E_NOCONV,)):
        x = torch.empty_like(b)
        info = PcgInfo()
        rc = self._check(lib().yasps_pcg(self.ctx, _ptr(b), _ptr(x), rtol, max_iter, C.byref(info)), allow)
        return x, dict(iters=info.iters, rel_residual=info.rel_residual, status=info.status, rc=rc)

    def pcg_noalloc(self, b, x, rtol=1e-8, max_iter=20000, allow=(E_NOCONV,)):
        """yasps_pcg_noalloc into a caller-provided x (no device allocation in the call)."""
        info = PcgInfo()
        rc = self._check(lib().yasps_pcg_noalloc(self.ctx, _ptr(b), _ptr(x), rtol, max_iter, C.byref(info)), allow)
        return dict(iters=info.iters, rel_residual=info.rel_residual, status=info.status, rc=rc)

    def newton_step(self, x, rtol=1e-8, max_iter=20000, max_halvings=40, armijo=1e-4, tie_rtol=0.0,
                    hessian=PROJECTED, shift=0.0, allow=(E_NOCONV,)):
        prm = NewtonParams(rtol, max_iter, max_halvings, armijo, tie_rtol, hessian, shift)
        info = NewtonInfo()
        rc = self._check(lib().yasps_newton_step(self.ctx, _ptr(x), C.byref(prm), C.byref(info)), allow)
        out = {k: getattr(info, k) for k, _ in NewtonInfo._fields_}
        out["status"] = rc
        return out

    def pattern(self, part):
        """Part 0 static (tets, triangles, hinges, bodies), 1 contacts, 2 body
        contacts: row_ptr, col_idx and the slot map (10 slots a stencil, 36 for
        part 2)."""
        n = self.n
        ns = (self.nt + self.nf + self.nh + self.nb, self.nc, self.nbc)[part]
        width = 36 if part == 2 else 10
        rp = np.zeros(n + 1, np.int32)
        self._check(lib().yasps_get_pattern(self.ctx, part, rp.ctypes.data_as(C.c_void_p), None, None))
        ci = np.zeros(max(int(rp[-1]), 1), np.int32)
        sl = np.zeros((max(ns, 1), width), np.int32)
        self._check(lib().yasps_get_pattern(self.ctx, part, rp.ctypes.data_as(C.c_void_p),
                                            ci.ctypes.data_as(C.c_void_p), sl.ctypes.data_as(C.c_void_p)))
        return rp, ci[:int(rp[-1])], sl[:ns]

    def spmv(self, x, y=None):
        y = torch.empty_like(x) if y is None else y
        self._check(lib().yasps_spmv(self.ctx, _ptr(x), _ptr(y)))
        return y

    def lm_shift(self, frac):
        """frac * median_v |tr(H_vv)| / (3 m_v) of the last assembly (yasps_lm_shift)."""
        out = C.c_double()
        self._check(lib().yasps_lm_shift(self.ctx, frac, C.byref(out)))
        return out.value

    def profile(self, enable=True):
        self._check(lib().yasps_profile_enable(self.ctx, int(bool(enable))))

    def profile_stats(self):
        out = {}
        for k, name in enumerate(KERNEL_CLASSES):
            n, ms = C.c_int32(), C.c_double()
            self._check(lib().yasps_profile_query(self.ctx, k, C.byref(n), C.byref(ms)))
            out[name] = dict(launches=n.value, total_ms=ms.value)
        return out

    def theta_adjoint(self, x, lam, theta):
        out = torch.empty(self.nt, dtype=torch.float64, device=self.dev)
        self._check(lib().yasps_theta_adjoint(self.ctx, _ptr(x), _ptr(lam), _ptr(theta), _ptr(out)))
        return out

    # ------------------------------------------------------------ time stepping
    def set_surface(self, points, edges, tris, edge_rest_len2=None, cell=None):
        """Host arrays: point ids (m,), edges (k, 2), triangles (t, 3), squared
        rest edge lengths (k,) or None, grid cell size (default: 1.01 x the
        longest rest edge)."""
        i32 = dict(dtype=torch.int32, device=self.dev)
        pts = torch.as_tensor(np.asarray(points, np.int32), **i32).contiguous()
        ed = torch.as_tensor(np.ascontiguousarray(np.asarray(edges, np.int32).reshape(-1, 2).T), **i32).contiguous()
        tr = torch.as_tensor(np.ascontiguousarray(np.asarray(tris, np.int32).reshape(-1, 3).T), **i32).contiguous()
        l2 = None
        if edge_rest_len2 is not None:
            l2 = torch.as_tensor(np.asarray(edge_rest_len2, np.float64), dtype=torch.float64, device=self.dev)
        if cell is None:
            cell = 1.01 * float(np.sqrt(np.max(edge_rest_len2))) if edge_rest_len2 is not None else 1.0
        S = Surface(int(pts.shape[0]), _ptr(pts), int(ed.shape[1]), _ptr(ed), int(tr.shape[1]), _ptr(tr), _ptr(l2),
                    float(cell))
        self._check(lib().yasps_set_surface(self.ctx, C.byref(S)))

    def detect(self, x):
        """Proximity search at x; the stencils become the contact set.  Returns
        (ctype (m,), cidx (m, 4), ee_eps (m,)) as host arrays."""
        n = C.c_int32()
        self._check(lib().yasps_detect(self.ctx, _ptr(x), C.byref(n)))
        m = n.value
        self.nc = m
        t = np.zeros(max(m, 1), np.int32)
        i = np.zeros((4, max(m, 1)), np.int32)
        e = np.zeros(max(m, 1), np.float64)
        self._check(lib().yasps_get_detected(self.ctx, t.ctypes.data_as(C.c_void_p), i.ctypes.data_as(C.c_void_p),
                                             e.ctypes.data_as(C.c_void_p)))
        return t[:m], np.ascontiguousarray(i.reshape(4, -1)[:, :m].T) if m else np.zeros((0, 4), np.int32), e[:m]

    def ccd(self, x, p, t_max=1.0, s=0.1):
        out = C.c_double()
        self._check(lib().yasps_ccd(self.ctx, _ptr(x), _ptr(p), t_max, s, C.byref(out)))
        return out.value

    def frame(self, x, v, tol=1e-2, max_newton=50, rtol=1e-8, max_iter=20000, armijo=1e-4, max_halvings=40,
              ccd_s=0.1, allow=()):
        prm = FrameParams(tol, max_newton, rtol, max_iter, armijo, max_halvings, ccd_s)
        info = FrameInfo()
        rc = self._check(lib().yasps_frame(self.ctx, _ptr(x), _ptr(v), C.byref(prm), C.byref(info)), allow)
        out = {k: getattr(info, k) for k, _ in FrameInfo._fields_}
        out["status"] = rc
        return out
