"""ctypes binding of libchebfilter.so: argument marshalling only.

Every entry point forwards to the C ABI declared in include/chebfilter.h; all
arithmetic runs in the library's HIP kernels.  Blocks are torch float64 CUDA
(HIP) tensors of shape [n, N] whose rows are contiguous (stride(1) == 1); the
row stride is passed as the leading dimension.  The library enqueues on the
torch stream that was current when the context was created.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libchebfilter.so")

CF_STATUS = {0: "CF_OK", 1: "CF_EINVAL", 2: "CF_ENOMEM", 3: "CF_ENOTSPD", 4: "CF_ENUMERIC",
             5: "CF_EDEVICE", 6: "CF_ENOTCONV"}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2}

EXPORTS = ["chebfilter_init", "chebfilter_destroy", "chebfilter_last_error", "chebfilter_sizes",
           "chebfilter_apply_H", "chebfilter_apply_M", "chebfilter_apply_Sinv",
           "chebfilter_filter", "chebfilter_filter_multipass", "chebfilter_cholqr",
           "chebfilter_rayleigh_ritz",
           "chebfilter_lanczos_bounds", "chebfilter_profile", "chebfilter_profile_query",
           "chebfilter_init_batch", "chebfilter_batch_destroy", "chebfilter_batch_last_error",
           "chebfilter_batch_sizes", "chebfilter_filter_batch", "chebfilter_rayleigh_ritz_batch",
           "chebfilter_lanczos_bounds_batch", "chebfilter_update_H_cc", "chebfilter_residual_norms",
           "chebfilter_mlp_create", "chebfilter_mlp_destroy", "chebfilter_mlp_last_error",
           "chebfilter_mlp_sizes", "chebfilter_mlp_set_params", "chebfilter_mlp_get_params",
           "chebfilter_mlp_forward", "chebfilter_mlp_loss_grad", "chebfilter_mlp_adam_step",
           "chebfilter_mlp_set_normalization", "chebfilter_bounds_features",
           "chebfilter_bounds_predict", "chebfilter_assembly_tables", "chebfilter_assemble_cells",
           "chebfilter_get_H_cc", "chebfilter_set_cell_tile", "chebfilter_autotune",
           "chebfilter_batch_autotune", "chebfilter_lanczos_bounds_noalloc", "chebfilter_tuning",
           "chebfilter_batch_tuning", "chebfilter_degree_rule", "chebfilter_step_summary",
           "chebfilter_bounds_label", "chebfilter_mlp_fit_normalization", "chebfilter_mlp_normalize",
           "chebfilter_mlp_predict", "chebfilter_enriched_tables", "chebfilter_adaptive_points",
           "chebfilter_assemble_enriched", "chebfilter_get_coupling", "chebfilter_scf_setup",
           "chebfilter_scf_sizes", "chebfilter_scf_geometry", "chebfilter_fermi_level",
           "chebfilter_scf_density", "chebfilter_scf_potential", "chebfilter_scf_assemble",
           "chebfilter_scf_mix", "chebfilter_scf_mix_reset"]


class CfProblem(C.Structure):
    _fields_ = [("p", C.c_int32), ("n_cells", C.c_int64), ("n_h", C.c_int64), ("n_e", C.c_int64),
                ("cell_dof", C.c_void_p), ("H_cc", C.c_void_p), ("M_cc_diag", C.c_void_p),
                ("enr_ptr", C.c_void_p), ("enr_idx", C.c_void_p), ("H_ec", C.c_void_p),
                ("M_ec", C.c_void_p), ("H_ee", C.c_void_p), ("M_ee", C.c_void_p)]


class CfOptions(C.Structure):
    _fields_ = [("device", C.c_int32), ("stream", C.c_void_p), ("max_cols", C.c_int64),
                ("col_chunk", C.c_int64), ("check_finite", C.c_int32)]


class CfAdaptiveGrid(C.Structure):
    _fields_ = [("ncells", C.c_int64), ("cells", C.c_void_p), ("cell_lo", C.c_void_p),
                ("h", C.c_double), ("n_nodes", C.c_int32), ("nodes", C.c_void_p),
                ("ng", C.c_int32), ("gauss_x", C.c_void_p), ("gauss_w", C.c_void_p),
                ("box_ptr", C.c_void_p), ("box_lo", C.c_void_p), ("box_size", C.c_void_p),
                ("n_atoms", C.c_int32), ("centers", C.c_void_p), ("n_shells", C.c_int32),
                ("shell_l", C.c_void_p), ("shell_term_ptr", C.c_void_p), ("term_c", C.c_void_p),
                ("term_k", C.c_void_p), ("term_zeta", C.c_void_p), ("r0", C.c_double),
                ("t", C.c_double)]


class CfScfSetup(C.Structure):
    _fields_ = [("cell_lo", C.c_void_p), ("plain_ref", C.c_void_p),
                ("comp_center", C.c_double * 3), ("comp_width", C.c_double),
                ("cg_max_iter", C.c_int32), ("cg_tol", C.c_double), ("mix_depth", C.c_int32),
                ("mix_beta", C.c_double)]


class ChebFilterError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{CF_STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load_library() -> C.CDLL:
    """Load the built library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1610_02121_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.chebfilter_init.argtypes = [C.POINTER(CfProblem), C.POINTER(CfOptions), C.POINTER(vp)]
    lib.chebfilter_destroy.argtypes = [vp]
    lib.chebfilter_last_error.argtypes = [vp]
    lib.chebfilter_last_error.restype = C.c_char_p
    lib.chebfilter_sizes.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    for nm in ("chebfilter_apply_H", "chebfilter_apply_M", "chebfilter_apply_Sinv"):
        getattr(lib, nm).argtypes = [vp, vp, i64, vp, i64, i64]
    lib.chebfilter_filter.argtypes = [vp, vp, i64, vp, i64, i64, i32, dbl, dbl, i32]
    lib.chebfilter_filter_multipass.argtypes = [vp, vp, i64, vp, i64, i64, i32, i32, dbl, dbl, i32]
    lib.chebfilter_cholqr.argtypes = [vp, vp, i64, i64]
    lib.chebfilter_rayleigh_ritz.argtypes = [vp, vp, i64, i64, vp]
    lib.chebfilter_lanczos_bounds.argtypes = [vp, vp, i32, C.POINTER(dbl), C.POINTER(dbl)]
    lib.chebfilter_lanczos_bounds_noalloc.argtypes = [vp, vp, i32, C.POINTER(dbl), C.POINTER(dbl)]
    lib.chebfilter_profile.argtypes = [vp, i32]
    lib.chebfilter_profile_query.argtypes = [vp, C.c_char_p, C.POINTER(i64), C.POINTER(dbl),
                                             C.POINTER(dbl)]
    P64 = C.POINTER(i64)
    lib.chebfilter_init_batch.argtypes = [C.POINTER(C.POINTER(CfProblem)), i32, C.POINTER(CfOptions),
                                          C.POINTER(vp)]
    lib.chebfilter_batch_destroy.argtypes = [vp]
    lib.chebfilter_batch_last_error.argtypes = [vp]
    lib.chebfilter_batch_last_error.restype = C.c_char_p
    lib.chebfilter_batch_sizes.argtypes = [vp, i32, P64, P64]
    lib.chebfilter_filter_batch.argtypes = [vp, C.POINTER(vp), P64, C.POINTER(vp), P64, P64, i32,
                                            C.POINTER(dbl), C.POINTER(dbl), i32, i32]
    lib.chebfilter_rayleigh_ritz_batch.argtypes = [vp, C.POINTER(vp), P64, P64, C.POINTER(vp)]
    lib.chebfilter_lanczos_bounds_batch.argtypes = [vp, C.POINTER(vp), i32, C.POINTER(dbl),
                                                    C.POINTER(dbl)]
    f32 = C.c_float
    PD = C.POINTER(dbl)
    lib.chebfilter_update_H_cc.argtypes = [vp, vp]
    lib.chebfilter_residual_norms.argtypes = [vp, vp, i64, i64, PD, PD]
    lib.chebfilter_mlp_create.argtypes = [i32, vp, i32, i32, i32, i32, i32, C.POINTER(vp)]
    lib.chebfilter_mlp_destroy.argtypes = [vp]
    lib.chebfilter_mlp_last_error.argtypes = [vp]
    lib.chebfilter_mlp_last_error.restype = C.c_char_p
    lib.chebfilter_mlp_sizes.argtypes = [vp, P64]
    lib.chebfilter_mlp_set_params.argtypes = [vp, vp, i32]
    lib.chebfilter_mlp_get_params.argtypes = [vp, vp]
    lib.chebfilter_mlp_forward.argtypes = [vp, vp, i32, vp]
    lib.chebfilter_mlp_loss_grad.argtypes = [vp, vp, vp, i32, C.POINTER(f32), vp]
    lib.chebfilter_mlp_adam_step.argtypes = [vp, f32, f32, f32, f32]
    lib.chebfilter_mlp_set_normalization.argtypes = [vp, PD, PD, PD, PD]
    lib.chebfilter_bounds_features.argtypes = [PD, i32, PD]
    lib.chebfilter_bounds_predict.argtypes = [vp, vp, PD, vp, i32, i32, i32, PD, PD,
                                              C.POINTER(i32), C.POINTER(i32)]
    lib.chebfilter_assembly_tables.argtypes = [vp, i32, vp, vp, vp]
    lib.chebfilter_assemble_cells.argtypes = [vp, vp, i64, vp, i64]
    lib.chebfilter_get_H_cc.argtypes = [vp, vp, i64, vp]
    lib.chebfilter_enriched_tables.argtypes = [vp, C.POINTER(CfAdaptiveGrid)]
    lib.chebfilter_adaptive_points.argtypes = [vp, P64]
    lib.chebfilter_assemble_enriched.argtypes = [vp, vp]
    lib.chebfilter_get_coupling.argtypes = [vp, vp, vp]
    lib.chebfilter_scf_setup.argtypes = [vp, C.POINTER(CfScfSetup)]
    lib.chebfilter_scf_sizes.argtypes = [vp, P64, P64]
    lib.chebfilter_scf_geometry.argtypes = [vp, vp, vp]
    lib.chebfilter_fermi_level.argtypes = [PD, i64, dbl, dbl, PD, PD]
    lib.chebfilter_scf_density.argtypes = [vp, vp, i64, i64, PD, vp]
    lib.chebfilter_scf_potential.argtypes = [vp, vp, vp, vp, PD, C.POINTER(i32)]
    lib.chebfilter_scf_assemble.argtypes = [vp, vp]
    lib.chebfilter_scf_mix.argtypes = [vp, vp, vp, vp, PD]
    lib.chebfilter_scf_mix_reset.argtypes = [vp]
    lib.chebfilter_set_cell_tile.argtypes = [vp, i32, i32]
    lib.chebfilter_autotune.argtypes = [vp, vp, i64, vp, i64, i64, i32, dbl, dbl, i32, i32,
                                        C.POINTER(i32)]
    lib.chebfilter_batch_autotune.argtypes = [vp, C.POINTER(vp), P64, C.POINTER(vp), P64, P64, i32,
                                              C.POINTER(dbl), C.POINTER(dbl), i32, i32,
                                              C.POINTER(i32)]
    lib.chebfilter_degree_rule.argtypes = [dbl, dbl, dbl, dbl, dbl, i32, i32, C.POINTER(i32)]
    lib.chebfilter_step_summary.argtypes = [PD, PD, i32, i32, dbl, i32, PD, PD]
    lib.chebfilter_bounds_label.argtypes = [vp, PD, i32, PD, i32, i32, vp, i32, i32, i32, PD, PD]
    lib.chebfilter_mlp_fit_normalization.argtypes = [vp, PD, PD, i64]
    lib.chebfilter_mlp_normalize.argtypes = [vp, i32, PD, i64, vp]
    lib.chebfilter_mlp_predict.argtypes = [vp, PD, i64, PD]
    lib.chebfilter_tuning.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.chebfilter_batch_tuning.argtypes = [vp, i32, C.POINTER(i32), C.POINTER(i32),
                                            C.POINTER(i32)]
    for nm in EXPORTS:
        if nm not in ("chebfilter_last_error", "chebfilter_batch_last_error",
                      "chebfilter_mlp_last_error"):
            getattr(lib, nm).restype = C.c_int
    _lib = lib
    return lib


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _block(t, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.dim() != 2 or (t.shape[1] > 1 and t.stride(1) != 1):
        raise ValueError(f"{name} must be 2-D with contiguous rows")
    return t.data_ptr(), t.stride(0) if t.shape[1] > 1 else max(t.stride(0), 1)


def empty_block(n: int, N: int, device, dtype=None):
    """An n x N device block whose leading dimension is N rounded up to a
    multiple of 16 (128 bytes of FP64): the row segments the kernels gather
    then start on cache-line boundaries.  Returns the [n, N] view."""
    import torch
    ld = (N + 15) // 16 * 16
    return torch.empty((n, ld), dtype=dtype or torch.float64, device=device)[:, :N]


def _problem_struct(prob):
    """(CfProblem, arrays it points into) for a synth Problem."""
    keep = {
        "cell_dof": _np(prob.cell_dof, np.int64), "H_cc": _np(prob.H_cc, np.float64),
        "M_cc_diag": _np(prob.M_cc_diag, np.float64), "enr_ptr": _np(prob.enr_ptr, np.int64),
        "enr_idx": _np(prob.enr_idx, np.int64), "H_ec": _np(prob.H_ec, np.float64),
        "M_ec": _np(prob.M_ec, np.float64), "H_ee": _np(prob.H_ee, np.float64),
        "M_ee": _np(prob.M_ee, np.float64)}
    n_cells = keep["cell_dof"].shape[0]
    cp = CfProblem(int(prob.p), n_cells, keep["M_cc_diag"].shape[0], keep["H_ee"].shape[0],
                   *[keep[f].ctypes.data for f in ("cell_dof", "H_cc", "M_cc_diag", "enr_ptr",
                                                   "enr_idx", "H_ec", "M_ec", "H_ee", "M_ee")])
    return cp, keep


def fermi_level(eps, n_electrons: float, kT: float):
    """(f, mu): occupations and Fermi level (chebfilter_fermi_level, Eq. FermiDirac / Mu)."""
    lib = load_library()
    e = _np(eps, np.float64).ravel()
    f = np.zeros_like(e)
    mu = C.c_double(0.0)
    PD = C.POINTER(C.c_double)
    st = lib.chebfilter_fermi_level(e.ctypes.data_as(PD), int(e.size), float(n_electrons),
                                    float(kT), f.ctypes.data_as(PD), C.byref(mu))
    if st != 0:
        raise ChebFilterError(st, "fermi_level: need 0 < n_electrons < 2 len(eps), kT > 0")
    return f, float(mu.value)


class Context:
    """One discrete problem resident on one GPU (wraps cf_ctx)."""

    def __init__(self, prob, max_cols: int, device: int = 0, check_finite: bool = False,
                 col_chunk: int = 0):
        import torch
        self.lib = load_library()
        cp, self._keep = _problem_struct(prob)
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        opt = CfOptions(device, C.c_void_p(stream.cuda_stream), int(max_cols), int(col_chunk),
                        int(check_finite))
        h = C.c_void_p()
        st = self.lib.chebfilter_init(C.byref(cp), C.byref(opt), C.byref(h))
        if st != 0:
            raise ChebFilterError(st, self.lib.chebfilter_last_error(None).decode())
        self._h = h
        self._keep = None
        nh, ne, mc = C.c_int64(), C.c_int64(), C.c_int64()
        self.lib.chebfilter_sizes(h, C.byref(nh), C.byref(ne), C.byref(mc))
        self.n_h, self.n_e, self.max_cols = nh.value, ne.value, mc.value
        self.n = self.n_h + self.n_e
        self._npc = (int(prob.p) + 1) ** 3
        self._nnz = int(np.asarray(prob.enr_ptr)[-1]) if self.n_e else 0

    def _check(self, st: int):
        if st != 0:
            raise ChebFilterError(st, self.lib.chebfilter_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.chebfilter_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out(self, X, Y):
        import torch
        if Y is None:
            Y = torch.empty_like(X)
        return Y

    def apply_H(self, X, Y=None):
        Y = self._out(X, Y)
        (xp, ldx), (yp, ldy) = _block(X, "X"), _block(Y, "Y")
        self._check(self.lib.chebfilter_apply_H(self._h, xp, ldx, yp, ldy, X.shape[1]))
        return Y

    def apply_M(self, X, Y=None):
        Y = self._out(X, Y)
        (xp, ldx), (yp, ldy) = _block(X, "X"), _block(Y, "Y")
        self._check(self.lib.chebfilter_apply_M(self._h, xp, ldx, yp, ldy, X.shape[1]))
        return Y

    def apply_Sinv(self, X, Y=None):
        Y = self._out(X, Y)
        (xp, ldx), (yp, ldy) = _block(X, "X"), _block(Y, "Y")
        self._check(self.lib.chebfilter_apply_Sinv(self._h, xp, ldx, yp, ldy, X.shape[1]))
        return Y

    def filter(self, X, m: int, a: float, b: float, Y=None, prec="fp64"):
        """Y = T_m(t(H~)) X; prec is "fp64", "fp32", "bf16" or a cf_prec code."""
        Y = self._out(X, Y)
        (xp, ldx), (yp, ldy) = _block(X, "X"), _block(Y, "Y")
        code = PREC[prec] if isinstance(prec, str) else int(prec)
        self._check(self.lib.chebfilter_filter(self._h, xp, ldx, yp, ldy, X.shape[1], int(m),
                                               float(a), float(b), code))
        return Y

    def filter_multipass(self, X, m: int, passes: int, a: float, b: float, Y=None, prec="fp64"):
        """passes x T_m(t(H~)) with Rayleigh-Ritz between the passes."""
        Y = self._out(X, Y)
        (xp, ldx), (yp, ldy) = _block(X, "X"), _block(Y, "Y")
        code = PREC[prec] if isinstance(prec, str) else int(prec)
        self._check(self.lib.chebfilter_filter_multipass(self._h, xp, ldx, yp, ldy, X.shape[1], int(m),
                                                         int(passes), float(a), float(b), code))
        return Y

    def set_cell_tile(self, prec: str, nsb: int):
        """Column blocks (1 or 2) per tile of the reduced cell product for the
        FP32-input ("fp32") or BF16-input ("bf16") cells."""
        self._check(self.lib.chebfilter_set_cell_tile(self._h, PREC[prec], int(nsb)))

    def autotune(self, X, m: int, a: float, b: float, prec="fp32", reps: int = 3, Y=None) -> int:
        """Time both tile shapes on this filter, keep the faster; returns it."""
        Y = self._out(X, Y)
        (xp, ldx), (yp, ldy) = _block(X, "X"), _block(Y, "Y")
        ch = C.c_int32(0)
        self._check(self.lib.chebfilter_autotune(self._h, xp, ldx, yp, ldy, X.shape[1], int(m),
                                                 float(a), float(b), PREC[prec], int(reps),
                                                 C.byref(ch)))
        return ch.value

    def tuning(self, coupling_map: int = -1) -> dict:
        """The tile-shape state (set the coupling map first if >= 0)."""
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.chebfilter_tuning(self._h, int(coupling_map), C.byref(a), C.byref(b),
                                               C.byref(c)))
        return {"nsb_fp32": a.value, "nsb_bf16": b.value, "coupling_map": c.value}

    def cholqr(self, Y):
        yp, ldy = _block(Y, "Y")
        self._check(self.lib.chebfilter_cholqr(self._h, yp, ldy, Y.shape[1]))
        return Y

    def rayleigh_ritz(self, Y) -> np.ndarray:
        yp, ldy = _block(Y, "Y")
        theta = np.zeros(max(Y.shape[1], 1), dtype=np.float64)
        self._check(self.lib.chebfilter_rayleigh_ritz(self._h, yp, ldy, Y.shape[1],
                                                      theta.ctypes.data))
        return theta[:Y.shape[1]]

    def lanczos_bounds(self, v0, k: int = 10) -> tuple[float, float]:
        import torch
        if v0.dtype != torch.float64 or not v0.is_cuda or not v0.is_contiguous():
            raise TypeError("v0 must be a contiguous float64 CUDA tensor")
        lo, hi = C.c_double(), C.c_double()
        self._check(self.lib.chebfilter_lanczos_bounds(self._h, v0.data_ptr(), int(k),
                                                       C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def lanczos_bounds_noalloc(self, v0, k: int = 10) -> tuple[float, float]:
        """lanczos_bounds with the library's fixed device scratch (no allocation)."""
        import torch
        if v0.dtype != torch.float64 or not v0.is_cuda or not v0.is_contiguous():
            raise TypeError("v0 must be a contiguous float64 CUDA tensor")
        lo, hi = C.c_double(), C.c_double()
        self._check(self.lib.chebfilter_lanczos_bounds_noalloc(self._h, v0.data_ptr(), int(k),
                                                               C.byref(lo), C.byref(hi)))
        return lo.value, hi.value

    def update_H_cc(self, H_cc):
        """Replace the elemental H^cc_e (host array [E, npc, npc])."""
        H = _np(H_cc, np.float64)
        self._check(self.lib.chebfilter_update_H_cc(self._h, H.ctypes.data))

    def assembly_tables(self, B, w, K):
        """Reference tables of the plain-cell quadrature: B [nq, npc] shape values,
        w [nq] weights with the Jacobian, K [npc, npc] kinetic block (host arrays)."""
        B, w, K = _np(B, np.float64), _np(w, np.float64), _np(K, np.float64)
        if B.ndim != 2 or w.shape != (B.shape[0],) or K.shape != (B.shape[1], B.shape[1]):
            raise ValueError("assembly_tables: B [nq, npc], w [nq], K [npc, npc]")
        self._check(self.lib.chebfilter_assembly_tables(self._h, int(B.shape[0]), B.ctypes.data,
                                                        w.ctypes.data, K.ctypes.data))

    def assemble_cells(self, cells, V):
        """H^cc_e = K + B^T diag(w V_e) B on the device for the listed plain
        cells; V is a float64 CUDA tensor [len(cells), nq] (row stride >= nq)."""
        import torch
        cl = _np(cells, np.int32)
        if V.dtype != torch.float64 or not V.is_cuda or V.dim() != 2 or V.stride(1) != 1:
            raise TypeError("V must be a float64 CUDA tensor [ncells, nq] with unit column stride")
        if V.shape[0] != cl.size:
            raise ValueError("V needs one row per cell")
        self._check(self.lib.chebfilter_assemble_cells(self._h, cl.ctypes.data, int(cl.size),
                                                       V.data_ptr(), int(V.stride(0))))

    def get_H_cc(self, cells) -> np.ndarray:
        """The current H^cc_e of the listed cells, [len(cells), npc, npc]."""
        cl = _np(cells, np.int32)
        out = np.zeros((cl.size, self._npc, self._npc))
        self._check(self.lib.chebfilter_get_H_cc(self._h, cl.ctypes.data, int(cl.size),
                                                 out.ctypes.data))
        return out

    def enriched_tables(self, cells, cell_lo, h, nodes, gauss_x, gauss_w, box_ptr, box_lo,
                        box_size, centers=None, shells=(), r0=1.0, t=1.0):
        """Upload the adaptive grid of the listed cells and the enrichment
        description (chebfilter_enriched_tables).  shells: [(l, [(c, k, zeta), ...])]
        per shell, the radial part as Slater-type terms.  Host arrays."""
        keep = [_np(cells, np.int32), _np(cell_lo, np.float64).reshape(-1, 3),
                _np(nodes, np.float64), _np(gauss_x, np.float64), _np(gauss_w, np.float64),
                _np(box_ptr, np.int64), _np(box_lo, np.float64).reshape(-1, 3),
                _np(box_size, np.float64)]
        cl, lo, nd, gx, gw, bp, bl, bs = keep
        cen = _np(centers if centers is not None else np.zeros((0, 3)), np.float64).reshape(-1, 3)
        sl = np.array([l for l, _ in shells], dtype=np.int32)
        tp = np.zeros(len(shells) + 1, dtype=np.int32)
        tc, tk, tz = [], [], []
        for s, (_, terms) in enumerate(shells):
            for c_, k_, z_ in terms:
                tc.append(c_)
                tk.append(k_)
                tz.append(z_)
            tp[s + 1] = len(tc)
        tc, tk, tz = (np.array(tc, dtype=np.float64), np.array(tk, dtype=np.int32),
                      np.array(tz, dtype=np.float64))
        keep += [cen, sl, tp, tc, tk, tz]
        g = CfAdaptiveGrid(ncells=cl.size, cells=cl.ctypes.data, cell_lo=lo.ctypes.data, h=float(h),
                           n_nodes=nd.size, nodes=nd.ctypes.data, ng=gx.size,
                           gauss_x=gx.ctypes.data, gauss_w=gw.ctypes.data, box_ptr=bp.ctypes.data,
                           box_lo=bl.ctypes.data, box_size=bs.ctypes.data, n_atoms=cen.shape[0],
                           centers=cen.ctypes.data, n_shells=sl.size, shell_l=sl.ctypes.data,
                           shell_term_ptr=tp.ctypes.data, term_c=tc.ctypes.data,
                           term_k=tk.ctypes.data, term_zeta=tz.ctypes.data, r0=float(r0),
                           t=float(t))
        self._check(self.lib.chebfilter_enriched_tables(self._h, C.byref(g)))

    def adaptive_points(self) -> int:
        """Points of the uploaded adaptive grid (length of assemble_enriched's V)."""
        n = C.c_int64(0)
        self._check(self.lib.chebfilter_adaptive_points(self._h, C.byref(n)))
        return int(n.value)

    def assemble_enriched(self, V):
        """Recompute H^cc_e, H^ec and H^ee of the listed cells on the device from
        the potential at the grid's points (float64 CUDA tensor [npoints])."""
        import torch
        if V.dtype != torch.float64 or not V.is_cuda or not V.is_contiguous():
            raise TypeError("V must be a contiguous float64 CUDA tensor")
        if V.numel() != self.adaptive_points():
            raise ValueError("V needs one value per point of the grid")
        self._check(self.lib.chebfilter_assemble_enriched(self._h, V.data_ptr()))

    def get_coupling(self):
        """The current H^ec [nnz, npc] (cf_problem.H_ec's layout) and H^ee
        [n_e, n_e] (host copies)."""
        Hec = np.zeros((self._nnz, self._npc))
        Hee = np.zeros((self.n_e, self.n_e))
        self._check(self.lib.chebfilter_get_coupling(self._h, Hec.ctypes.data, Hee.ctypes.data))
        return Hec, Hee

    # ---- self-consistent field quantities
    def scf_setup(self, cell_lo, plain_ref, comp_center, comp_width, cg_max_iter: int = 4000,
                  cg_tol: float = 1e-11, mix_depth: int = 4, mix_beta: float = 0.5):
        """Points, Poisson system and mixing state (chebfilter_scf_setup)."""
        lo = _np(cell_lo, np.float64).reshape(-1, 3)
        ref = _np(plain_ref, np.float64).reshape(-1, 3)
        st = CfScfSetup(cell_lo=lo.ctypes.data, plain_ref=ref.ctypes.data,
                        comp_center=(C.c_double * 3)(*[float(x) for x in comp_center]),
                        comp_width=float(comp_width), cg_max_iter=int(cg_max_iter),
                        cg_tol=float(cg_tol), mix_depth=int(mix_depth), mix_beta=float(mix_beta))
        self._check(self.lib.chebfilter_scf_setup(self._h, C.byref(st)))
        P, Pp = C.c_int64(), C.c_int64()
        self._check(self.lib.chebfilter_scf_sizes(self._h, C.byref(P), C.byref(Pp)))
        self.scf_points, self.scf_plain_points = int(P.value), int(Pp.value)

    def scf_geometry(self):
        """(xyz [P, 3], w [P]) of the SCF points (host copies)."""
        xyz = np.zeros((self.scf_points, 3))
        w = np.zeros(self.scf_points)
        self._check(self.lib.chebfilter_scf_geometry(self._h, xyz.ctypes.data, w.ctypes.data))
        return xyz, w

    def _field(self, name, t):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() \
                or t.numel() != self.scf_points:
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor of one value per point")

    def scf_density(self, X, f):
        """rho at the points (Eq. Rho) of the block X [n, N] with occupations f [N]."""
        import torch
        xp, ldx = _block(X, "X")
        if X.shape[0] != self.n:
            raise ValueError("X needs one row per DOF")
        ff = _np(f, np.float64).ravel()
        if ff.size != X.shape[1]:
            raise ValueError("one occupation per column")
        rho = torch.empty(self.scf_points, dtype=torch.float64, device=self.device)
        PD = C.POINTER(C.c_double)
        self._check(self.lib.chebfilter_scf_density(self._h, xp, int(ldx), int(X.shape[1]),
                                                    ff.ctypes.data_as(PD), rho.data_ptr()))
        return rho

    def scf_potential(self, rho, v_ext):
        """(V_eff [P] tensor, terms dict, CG iterations): LDA, Poisson, sum."""
        import torch
        self._field("rho", rho)
        self._field("v_ext", v_ext)
        veff = torch.empty_like(rho)
        terms = np.zeros(5)
        it = C.c_int32(0)
        PD = C.POINTER(C.c_double)
        self._check(self.lib.chebfilter_scf_potential(self._h, rho.data_ptr(), v_ext.data_ptr(),
                                                      veff.data_ptr(), terms.ctypes.data_as(PD),
                                                      C.byref(it)))
        names = ("charge", "E_xc", "int_rho_vxc", "half_int_rho_vh", "cg_rel_residual")
        return veff, dict(zip(names, map(float, terms))), int(it.value)

    def scf_assemble(self, v_eff):
        """H blocks of every cell from V_eff at the points."""
        self._field("v_eff", v_eff)
        self._check(self.lib.chebfilter_scf_assemble(self._h, v_eff.data_ptr()))

    def scf_mix(self, rho_in, rho_out):
        """(rho_next, ||rho_out - rho_in||_w) by n-stage Anderson mixing."""
        import torch
        self._field("rho_in", rho_in)
        self._field("rho_out", rho_out)
        nxt = torch.empty_like(rho_in)
        r = C.c_double(0.0)
        self._check(self.lib.chebfilter_scf_mix(self._h, rho_in.data_ptr(), rho_out.data_ptr(),
                                                nxt.data_ptr(), C.byref(r)))
        return nxt, float(r.value)

    def scf_mix_reset(self):
        self._check(self.lib.chebfilter_scf_mix_reset(self._h))

    def bounds_label(self, history, theta, wanted: int, v0, k: int = 40, m_min: int = 8,
                     m_max: int = 120):
        """(input, target) training sample for the current operator (chebfilter_bounds_label)."""
        h = _np(history, np.float64).ravel()
        th = _np(theta, np.float64)
        inp, tgt = np.zeros(h.size), np.zeros(3)
        PD = C.POINTER(C.c_double)
        self._check(self.lib.chebfilter_bounds_label(
            self._h, h.ctypes.data_as(PD), h.size // 8, th.ctypes.data_as(PD), int(th.size),
            int(wanted), v0.data_ptr(), int(k), int(m_min), int(m_max), inp.ctypes.data_as(PD),
            tgt.ctypes.data_as(PD)))
        return inp, tgt

    def residual_norms(self, Z, theta) -> np.ndarray:
        """||H z_j - theta_j M z_j||_{M^-1} per column of Z."""
        zp, ldz = _block(Z, "Z")
        N = Z.shape[1]
        th = _np(theta, np.float64)[:N]
        res = np.zeros(max(N, 1))
        self._check(self.lib.chebfilter_residual_norms(
            self._h, zp, ldz, N, th.ctypes.data_as(C.POINTER(C.c_double)),
            res.ctypes.data_as(C.POINTER(C.c_double))))
        return res[:N]

    def bounds_predict(self, mlp, history, v0, lanczos_k: int = 10, m_min: int = 8,
                       m_max: int = 120):
        """(a, b, m, used_lanczos) for the next filter from the network and the guard."""
        import torch
        if v0.dtype != torch.float64 or not v0.is_cuda or not v0.is_contiguous():
            raise TypeError("v0 must be a contiguous float64 CUDA tensor")
        h = _np(history, np.float64).ravel()
        a, b = C.c_double(), C.c_double()
        m, fb = C.c_int32(), C.c_int32()
        self._check(self.lib.chebfilter_bounds_predict(
            self._h, mlp._h, h.ctypes.data_as(C.POINTER(C.c_double)), v0.data_ptr(), int(lanczos_k),
            int(m_min), int(m_max), C.byref(a), C.byref(b), C.byref(m), C.byref(fb)))
        return a.value, b.value, m.value, bool(fb.value)

    def profile(self, enable: bool):
        self._check(self.lib.chebfilter_profile(self._h, int(enable)))

    def profile_query(self, name: str) -> tuple[int, float, float]:
        """(launches, total milliseconds, total algorithmic flops) of a kernel family."""
        n, ms, fl = C.c_int64(), C.c_double(), C.c_double()
        self._check(self.lib.chebfilter_profile_query(self._h, name.encode(), C.byref(n),
                                                      C.byref(ms), C.byref(fl)))
        return n.value, ms.value, fl.value


class Batch:
    """Independent problems filtered together (wraps cf_batch).  The same
    Problem object appearing several times shares one device operator."""

    def __init__(self, probs, max_cols: int, device: int = 0):
        import torch
        self.lib = load_library()
        structs, keep, index = [], [], {}
        ptrs = (C.POINTER(CfProblem) * len(probs))()
        for i, p in enumerate(probs):
            if id(p) not in index:
                cp, arrs = _problem_struct(p)
                structs.append(cp)
                keep.append(arrs)
                index[id(p)] = len(structs) - 1
            ptrs[i] = C.pointer(structs[index[id(p)]])
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        opt = CfOptions(device, C.c_void_p(stream.cuda_stream), int(max_cols), 0, 0)
        h = C.c_void_p()
        st = self.lib.chebfilter_init_batch(ptrs, len(probs), C.byref(opt), C.byref(h))
        if st != 0:
            raise ChebFilterError(st, self.lib.chebfilter_batch_last_error(None).decode())
        self._h = h
        self.count = len(probs)
        self.max_cols = int(max_cols)
        self.sizes = []
        for i in range(self.count):
            nh, ne = C.c_int64(), C.c_int64()
            self.lib.chebfilter_batch_sizes(h, i, C.byref(nh), C.byref(ne))
            self.sizes.append((nh.value, ne.value))

    def _check(self, st: int):
        if st != 0:
            raise ChebFilterError(st, self.lib.chebfilter_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.chebfilter_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _blocks(self, blocks, name):
        n = self.count
        if len(blocks) != n:
            raise ValueError(f"{name}: need {n} blocks")
        ptrs, lds, Ns = (C.c_void_p * n)(), (C.c_int64 * n)(), (C.c_int64 * n)()
        for i, t in enumerate(blocks):
            p, ld = _block(t, f"{name}[{i}]")
            ptrs[i], lds[i], Ns[i] = p, ld, t.shape[1]
        return ptrs, lds, Ns

    def filter(self, X, m: int, a, b, Y=None, prec="fp32", use_graph: bool = True):
        """Y[i] = T_m(t_i(H~_i)) X[i] for every entry (lists of blocks, a, b)."""
        import torch
        if Y is None:
            Y = [torch.empty_like(x) for x in X]
        xp, xl, xn = self._blocks(X, "X")
        yp, yl, yn = self._blocks(Y, "Y")
        if list(xn) != list(yn):
            raise ValueError("X and Y column counts differ")
        n = self.count
        av = (C.c_double * n)(*[float(v) for v in a])
        bv = (C.c_double * n)(*[float(v) for v in b])
        code = PREC[prec] if isinstance(prec, str) else int(prec)
        self._check(self.lib.chebfilter_filter_batch(self._h, xp, xl, yp, yl, xn, int(m), av, bv,
                                                     code, int(bool(use_graph))))
        return Y

    def autotune(self, X, m: int, a, b, prec="fp32", reps: int = 3, Y=None) -> int:
        """Time both tile shapes of the batched reduced cell product on this
        batched filter, keep the faster; returns it."""
        import torch
        if Y is None:
            Y = [torch.empty_like(x) for x in X]
        xp, xl, xn = self._blocks(X, "X")
        yp, yl, yn = self._blocks(Y, "Y")
        n = self.count
        av = (C.c_double * n)(*[float(v) for v in a])
        bv = (C.c_double * n)(*[float(v) for v in b])
        ch = C.c_int32(0)
        self._check(self.lib.chebfilter_batch_autotune(self._h, xp, xl, yp, yl, xn, int(m), av, bv,
                                                       PREC[prec], int(reps), C.byref(ch)))
        return ch.value

    def tuning(self, coupling_map: int = -1) -> dict:
        """The batch's tile-shape state (set the coupling map first if >= 0)."""
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.chebfilter_batch_tuning(self._h, int(coupling_map), C.byref(a),
                                                     C.byref(b), C.byref(c)))
        return {"nsb_fp32": a.value, "nsb_bf16": b.value, "coupling_map": c.value}

    def rayleigh_ritz(self, Y):
        yp, yl, yn = self._blocks(Y, "Y")
        thetas = [np.zeros(max(int(N), 1)) for N in yn]
        tp = (C.c_void_p * self.count)(*[t.ctypes.data for t in thetas])
        self._check(self.lib.chebfilter_rayleigh_ritz_batch(self._h, yp, yl, yn, tp))
        return [t[:int(N)] for t, N in zip(thetas, yn)]

    def lanczos_bounds(self, v0, k: int = 10):
        import torch
        n = self.count
        vp = (C.c_void_p * n)()
        for i, v in enumerate(v0):
            if v.dtype != torch.float64 or not v.is_cuda or not v.is_contiguous():
                raise TypeError("v0 entries must be contiguous float64 CUDA tensors")
            vp[i] = v.data_ptr()
        lo, hi = (C.c_double * n)(), (C.c_double * n)()
        self._check(self.lib.chebfilter_lanczos_bounds_batch(self._h, vp, int(k), lo, hi))
        return list(lo), list(hi)


def bounds_features(history) -> np.ndarray:
    """Scale-free network inputs of a raw history (chebfilter_bounds_features)."""
    lib = load_library()
    h = _np(history, np.float64).ravel()
    out = np.zeros_like(h)
    st = lib.chebfilter_bounds_features(h.ctypes.data_as(C.POINTER(C.c_double)), h.size // 8,
                                        out.ctypes.data_as(C.POINTER(C.c_double)))
    if st != 0:
        raise ChebFilterError(st, "bounds_features: the last step's b - theta_N must be > 0")
    return out


def degree_rule(theta_1: float, theta_w: float, a: float, b: float, rho: float = 100.0,
                m_min: int = 8, m_max: int = 120) -> int:
    """chebfilter_degree_rule."""
    lib = load_library()
    m = C.c_int32()
    st = lib.chebfilter_degree_rule(float(theta_1), float(theta_w), float(a), float(b), float(rho),
                                    int(m_min), int(m_max), C.byref(m))
    if st != 0:
        raise ChebFilterError(st, "degree_rule: need b > a, rho > 1, 1 <= m_min <= m_max")
    return m.value


def step_summary(theta, theta_prev, wanted: int, b_used: float, m_used: int, res) -> np.ndarray:
    """chebfilter_step_summary: the 8 raw features of one step."""
    lib = load_library()
    th, tp, r = _np(theta, np.float64), _np(theta_prev, np.float64), _np(res, np.float64)
    out = np.zeros(8)
    PD = C.POINTER(C.c_double)
    st = lib.chebfilter_step_summary(th.ctypes.data_as(PD), tp.ctypes.data_as(PD), int(th.size),
                                     int(wanted), float(b_used), int(m_used), r.ctypes.data_as(PD),
                                     out.ctypes.data_as(PD))
    if st != 0:
        raise ChebFilterError(st, "step_summary: bad sizes")
    return out


class Mlp:
    """The bounds network on the GPU (wraps cf_mlp): FP32 parameters, forward,
    mean-squared-error gradient and Adam, all in the library's kernels."""

    def __init__(self, n_in: int, width: int, depth: int, n_out: int, max_batch: int,
                 device: int = 0):
        import torch
        self.lib = load_library()
        self.device = torch.device("cuda", device)
        stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        st = self.lib.chebfilter_mlp_create(device, C.c_void_p(stream.cuda_stream), n_in, width, depth,
                                            n_out, max_batch, C.byref(h))
        if st != 0:
            raise ChebFilterError(st, self.lib.chebfilter_mlp_last_error(None).decode())
        self._h = h
        self.n_in, self.width, self.depth, self.n_out = n_in, width, depth, n_out
        self.max_batch = max_batch
        npar = C.c_int64()
        self.lib.chebfilter_mlp_sizes(h, C.byref(npar))
        self.nparams = npar.value

    def _check(self, st: int):
        if st != 0:
            raise ChebFilterError(st, self.lib.chebfilter_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.chebfilter_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params, reset_adam: bool = True):
        p = _np(params, np.float32)
        if p.size != self.nparams:
            raise ValueError(f"need {self.nparams} parameters")
        self._check(self.lib.chebfilter_mlp_set_params(self._h, p.ctypes.data, int(reset_adam)))

    def get_params(self) -> np.ndarray:
        p = np.zeros(self.nparams, dtype=np.float32)
        self._check(self.lib.chebfilter_mlp_get_params(self._h, p.ctypes.data))
        return p

    @staticmethod
    def _dev32(t, name):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda \
                or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
        return t.data_ptr()

    def forward(self, X):
        import torch
        Y = torch.empty((X.shape[0], self.n_out), dtype=torch.float32, device=X.device)
        self._check(self.lib.chebfilter_mlp_forward(self._h, self._dev32(X, "X"), X.shape[0],
                                                    Y.data_ptr()))
        return Y

    def loss_grad(self, X, T, want_grad: bool = False):
        loss = C.c_float()
        g = np.zeros(self.nparams, dtype=np.float32) if want_grad else None
        self._check(self.lib.chebfilter_mlp_loss_grad(
            self._h, self._dev32(X, "X"), self._dev32(T, "T"), X.shape[0], C.byref(loss),
            g.ctypes.data if want_grad else None))
        return (loss.value, g) if want_grad else loss.value

    def adam_step(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self._check(self.lib.chebfilter_mlp_adam_step(self._h, lr, beta1, beta2, eps))

    def fit_normalization(self, inputs, targets):
        """chebfilter_mlp_fit_normalization on a corpus [count, n_in], [count, n_out]."""
        x, t = _np(inputs, np.float64), _np(targets, np.float64)
        PD = C.POINTER(C.c_double)
        self._check(self.lib.chebfilter_mlp_fit_normalization(self._h, x.ctypes.data_as(PD),
                                                              t.ctypes.data_as(PD), int(x.shape[0])))

    def _normalized(self, which: int, x):
        import torch
        x = _np(x, np.float64)
        out = np.zeros(x.shape, dtype=np.float32)
        self._check(self.lib.chebfilter_mlp_normalize(
            self._h, which, x.ctypes.data_as(C.POINTER(C.c_double)), int(x.shape[0]),
            out.ctypes.data))
        return torch.tensor(out, device=self.device)

    def normalize_inputs(self, inputs):
        """Inputs [count, n_in] normalised by the library, as an FP32 device tensor."""
        return self._normalized(0, inputs)

    def normalize_targets(self, targets):
        """Targets [count, n_out] normalised by the library, as an FP32 device tensor."""
        return self._normalized(1, targets)

    def predict(self, inputs) -> np.ndarray:
        """Raw outputs [count, n_out] of raw inputs (chebfilter_mlp_predict)."""
        x = _np(inputs, np.float64)
        y = np.zeros((x.shape[0], self.n_out))
        PD = C.POINTER(C.c_double)
        self._check(self.lib.chebfilter_mlp_predict(self._h, x.ctypes.data_as(PD), int(x.shape[0]),
                                                    y.ctypes.data_as(PD)))
        return y

    def set_normalization(self, in_mean, in_std, out_mean, out_std):
        arrs = [_np(v, np.float64) for v in (in_mean, in_std, out_mean, out_std)]
        self._keep_norm = arrs
        self._check(self.lib.chebfilter_mlp_set_normalization(
            self._h, *[a.ctypes.data_as(C.POINTER(C.c_double)) for a in arrs]))
