"""Python binding of libtefmm.so (argument marshalling only).

Every step of the evaluation runs in the library's HIP kernels; PyTorch is
used for device memory and streams.  Importing this module does not load the
library; the first call does, and raises if libtefmm.so is missing (run
``python -m paper_1902_05875_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtefmm.so")

TEFMM_FP64, TEFMM_MIXED_FP32 = 0, 1
MAX_LAYERS = 8  # TEFMM_MAX_LAYERS
TEFMM_NORM_PHYSICAL, TEFMM_NORM_PAPER = 0, 1
TEFMM_SIGMA_IMAGES, TEFMM_SIGMA_SOMMERFELD = 0, 1
SIGMA_TABLES = {"images": TEFMM_SIGMA_IMAGES, "sommerfeld": TEFMM_SIGMA_SOMMERFELD}
ERRORS = {0: "OK", -1: "INVALID_ARG", -2: "PARTICLE_ON_INTERFACE", -3: "UNSUPPORTED", -4: "HIP",
          -5: "DCIM_FIT", -6: "OOM", -7: "STATE"}

EXPORTS = ["tefmm_default_options", "tefmm_create", "tefmm_set_particles", "tefmm_evaluate",
           "tefmm_get_stats", "tefmm_last_error", "tefmm_destroy", "tefmm_densities",
           "tefmm_dcim_family", "tefmm_taylor_coefficients", "tefmm_get_moments", "tefmm_get_tree",
           "tefmm_selftest_mfma", "tefmm_evaluate_batch", "tefmm_autotune", "tefmm_dcim_cross",
           "tefmm_mlp_create", "tefmm_mlp_destroy", "tefmm_mlp_num_params", "tefmm_mlp_last_error",
           "tefmm_mlp_set_params", "tefmm_mlp_get_params", "tefmm_mlp_set_split", "tefmm_mlp_forward", "tefmm_mlp_forward_noalloc",
           "tefmm_mlp_loss_grad",
           "tefmm_mlp_adam_step", "tefmm_mlp_train", "tefmm_surrogate_default_options", "tefmm_surrogate_train",
           "tefmm_surrogate_destroy", "tefmm_surrogate_cell_ok", "tefmm_set_surrogate", "tefmm_surrogate_cell_errors",
           "tefmm_reset_timers", "tefmm_set_allocator", "tefmm_gmres", "tefmm_sigma_derivatives",
           "tefmm_radix_sort", "tefmm_exclusive_scan", "tefmm_evaluate_batch_queue", "tefmm_batch_check",
           "tefmm_sym_derivatives", "tefmm_sym_m2l", "tefmm_delta_derivatives", "tefmm_cross_derivatives"]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """Device memory of a handle from PyTorch's caching allocator (tefmm_set_allocator):
    blocks are taken on the current stream and returned to torch's cache."""

    def __init__(self):
        import torch
        self._torch = torch

        def _alloc(nbytes, user):
            try:
                return self._torch.cuda.caching_allocator_alloc(int(nbytes))
            except Exception:  # out of memory: NULL tells the library
                return None

        def _free(ptr, user):
            self._torch.cuda.caching_allocator_delete(ptr)

        self.alloc = ALLOC_FN(_alloc)  # kept alive as long as the handle uses them
        self.free = FREE_FN(_free)


class TefmmError(RuntimeError):
    def __init__(self, code, msg=""):
        super().__init__(f"tefmm error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class MediumC(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int), ("interfaces", ctypes.POINTER(ctypes.c_double)),
                ("k", ctypes.POINTER(ctypes.c_double))]


class OptionsC(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int), ("depth", ctypes.c_int), ("max_leaf", ctypes.c_int),
                ("precision", ctypes.c_int), ("normalization", ctypes.c_int), ("dcim_T1", ctypes.c_double),
                ("dcim_samples", ctypes.c_int), ("dcim_svd_tol", ctypes.c_double),
                ("interface_eps", ctypes.c_double), ("n_rhs_max", ctypes.c_int), ("dcim_T1_cross", ctypes.c_double),
                ("m2l_tile", ctypes.c_int), ("p2p_targets", ctypes.c_int), ("p2p_poly", ctypes.c_int),
                ("sigma_tables", ctypes.c_int)]


class StatsC(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ["t_setup_tree_ms", "t_setup_tables_ms", "t_setup_dcim_ms", "t_p2m_ms", "t_m2m_ms", "t_m2l_ms",
                 "t_l2l_ms", "t_l2p_ms", "t_p2p_ms", "t_total_ms"]] + [
        ("m2l_pairs", ctypes.c_int64), ("p2p_pairs", ctypes.c_int64), ("n_images", ctypes.c_int * (3 * MAX_LAYERS)),
        ("dcim_fit_err", ctypes.c_double * (3 * MAX_LAYERS)), ("depth", ctypes.c_int * MAX_LAYERS),
        ("n_families", ctypes.c_int),
        ("m2l_flops", ctypes.c_double), ("m2l_launches", ctypes.c_int), ("n_rhs", ctypes.c_int),
        ("cross_pairs", ctypes.c_int64), ("cross_pairs_forced", ctypes.c_int64), ("n_cross_fits", ctypes.c_int),
        ("cross_fit_err", ctypes.c_double), ("sigma_keys", ctypes.c_int64), ("surrogate_keys", ctypes.c_int64),
        ("timed_evaluations", ctypes.c_int), ("p2p_pairs_same_leaf", ctypes.c_int64),
        ("p2p_poly_err", ctypes.c_double), ("sigma_direct_pairs", ctypes.c_int64),
        ("occupied_leaves", ctypes.c_int64), ("max_leaf_count", ctypes.c_int64),
        ("reaction_keys_forced", ctypes.c_int64), ("sigma_quad_nodes", ctypes.c_int64),
        ("sigma_quad_keys", ctypes.c_int64)]


class GmresInfoC(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("matvecs", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("converged", ctypes.c_int)]


class SurOptionsC(ctypes.Structure):
    _fields_ = [("layer", ctypes.c_int), ("rho_max", ctypes.c_double), ("s_lo", ctypes.c_double),
                ("s_hi", ctypes.c_double), ("n_train", ctypes.c_int), ("epochs", ctypes.c_int),
                ("batch", ctypes.c_int), ("lr", ctypes.c_float), ("width", ctypes.c_int), ("n_hidden", ctypes.c_int),
                ("cells_rho", ctypes.c_int), ("cells_s", ctypes.c_int), ("n_valid", ctypes.c_int),
                ("budget", ctypes.c_double), ("seed", ctypes.c_uint64), ("h_from_images", ctypes.c_int),
                ("envelope", ctypes.c_int), ("leaf_level", ctypes.c_int), ("split_bf16", ctypes.c_int),
                ("err_total", ctypes.c_double)]


class SurReportC(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("t_data_s", ctypes.c_double), ("t_train_s", ctypes.c_double),
                ("t_valid_s", ctypes.c_double), ("final_loss", ctypes.c_double), ("max_cell_err", ctypes.c_double),
                ("cells_ok", ctypes.c_int), ("cells_total", ctypes.c_int), ("n_out", ctypes.c_int),
                ("n_params", ctypes.c_int64)]


_lib = None


def lib():
    """Load libtefmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1902_05875_amd.build")
        # torch must own the process's HIP runtime (libamdhip64.so.7): loading it first makes the
        # library bind to the same runtime, so torch's streams and allocations are valid here
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.tefmm_default_options.argtypes = [ctypes.POINTER(OptionsC)]
        L.tefmm_default_options.restype = None
        L.tefmm_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(MediumC), ctypes.POINTER(OptionsC)]
        L.tefmm_set_particles.argtypes = [vp, i64, vp, i32, vp]
        L.tefmm_evaluate.argtypes = [vp, vp, i32, vp, vp]
        L.tefmm_get_stats.argtypes = [vp, ctypes.POINTER(StatsC)]
        L.tefmm_last_error.argtypes = [vp]
        L.tefmm_last_error.restype = ctypes.c_char_p
        L.tefmm_destroy.argtypes = [vp]
        L.tefmm_destroy.restype = None
        L.tefmm_densities.argtypes = [ctypes.POINTER(MediumC), i32, i32, vp, vp]
        L.tefmm_dcim_family.argtypes = [ctypes.POINTER(MediumC), ctypes.POINTER(OptionsC), i32, i32, dbl, dbl,
                                        i32, ctypes.POINTER(i32), vp, vp, ctypes.POINTER(dbl)]
        L.tefmm_taylor_coefficients.argtypes = [i32, vp, vp, vp, dbl, dbl, i32, vp]
        L.tefmm_get_moments.argtypes = [vp, i32, i32, vp, i64]
        L.tefmm_get_tree.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, ctypes.POINTER(dbl)]
        L.tefmm_selftest_mfma.argtypes = []
        L.tefmm_evaluate_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), ctypes.POINTER(i32),
                                           ctypes.POINTER(vp), vp]
        L.tefmm_evaluate_batch_queue.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp),
                                                 ctypes.POINTER(i32), ctypes.POINTER(vp), vp]
        L.tefmm_batch_check.argtypes = [vp, vp]
        L.tefmm_sym_derivatives.argtypes = [dbl, i32, i64, vp, vp, vp]
        L.tefmm_sym_m2l.argtypes = [dbl, i32, i64, vp, vp, vp, vp]
        L.tefmm_autotune.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.tefmm_dcim_cross.argtypes = [ctypes.POINTER(MediumC), ctypes.POINTER(OptionsC), i32, i32, i32, dbl, i32,
                                       dbl, dbl, i32, ctypes.POINTER(i32), vp, vp, ctypes.POINTER(dbl)]
        L.tefmm_mlp_create.argtypes = [ctypes.POINTER(vp), i32, i32, i32, i32, ctypes.c_uint64]
        L.tefmm_mlp_destroy.argtypes = [vp]
        L.tefmm_mlp_destroy.restype = None
        L.tefmm_mlp_num_params.argtypes = [vp]
        L.tefmm_mlp_num_params.restype = i64
        L.tefmm_mlp_last_error.argtypes = [vp]
        L.tefmm_mlp_last_error.restype = ctypes.c_char_p
        L.tefmm_mlp_set_params.argtypes = [vp, vp]
        L.tefmm_mlp_get_params.argtypes = [vp, vp]
        L.tefmm_mlp_set_split.argtypes = [vp, i32]
        L.tefmm_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
        L.tefmm_mlp_forward_noalloc.argtypes = [vp, vp, i64, vp, vp]
        L.tefmm_mlp_loss_grad.argtypes = [vp, vp, vp, i64, ctypes.POINTER(dbl), vp, vp]
        L.tefmm_mlp_adam_step.argtypes = [vp, ctypes.c_float, vp]
        L.tefmm_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_float, ctypes.c_uint64, vp, vp]
        L.tefmm_surrogate_default_options.argtypes = [ctypes.POINTER(MediumC), i32, ctypes.POINTER(SurOptionsC)]
        L.tefmm_surrogate_default_options.restype = None
        L.tefmm_surrogate_train.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(MediumC), ctypes.POINTER(OptionsC),
                                            ctypes.POINTER(SurOptionsC), ctypes.POINTER(SurReportC), vp, vp]
        L.tefmm_surrogate_destroy.argtypes = [vp]
        L.tefmm_surrogate_destroy.restype = None
        L.tefmm_surrogate_cell_ok.argtypes = [vp, i32, vp, vp]
        L.tefmm_set_surrogate.argtypes = [vp, vp]
        L.tefmm_surrogate_cell_errors.argtypes = [vp, vp]
        L.tefmm_reset_timers.argtypes = [vp]
        L.tefmm_set_allocator.argtypes = [vp, ALLOC_FN, FREE_FN, vp]
        L.tefmm_gmres.argtypes = [vp, dbl, dbl, vp, vp, i32, i32, i32, dbl, vp, ctypes.POINTER(GmresInfoC)]
        L.tefmm_sigma_derivatives.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp]
        L.tefmm_delta_derivatives.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp]
        L.tefmm_cross_derivatives.argtypes = [vp, i32, i32, i32, i64, vp, vp, vp, vp, vp]
        L.tefmm_radix_sort.argtypes = [i64, vp, vp, i32, vp]
        L.tefmm_exclusive_scan.argtypes = [i64, vp, vp, vp]
        _lib = L
    return _lib


def radix_sort(keys, vals, end_bit, stream=None):
    """Stable in-place sort of device int32 tensors (keys read as unsigned) by the key bits
    [0, end_bit) (tefmm_radix_sort)."""
    _check(lib().tefmm_radix_sort(keys.numel(), keys.data_ptr(), vals.data_ptr(), int(end_bit), _stream_ptr(stream)))


def exclusive_scan(x, out, stream=None):
    """out = exclusive prefix sums of the device int32 tensor x, unsigned 32-bit
    arithmetic (tefmm_exclusive_scan)."""
    _check(lib().tefmm_exclusive_scan(x.numel(), x.data_ptr(), out.data_ptr(), _stream_ptr(stream)))


def sym_derivatives(k, order, R, stream=None):
    """D^s_{nm} h0(k|R|) for n <= order at the displacements R ((n, 3) array): numpy
    (n, C(order+3,3)) complex128 (tefmm_sym_derivatives, Theorem 4.2)."""
    import numpy as np
    R = np.ascontiguousarray(R, np.float64).reshape(-1, 3)
    cnt = (order + 1) * (order + 2) * (order + 3) // 6
    out = np.empty((R.shape[0], cnt), np.complex128)
    _check(lib().tefmm_sym_derivatives(float(k), int(order), R.shape[0], R.ctypes.data, out.ctypes.data,
                                        _stream_ptr(stream)))
    return out


def sym_m2l(k, p, R, alpha, stream=None):
    """TEFMM-II translation of Eq. M2Ltransop (tefmm_sym_m2l): R (n, 3) displacements (host),
    alpha a (n, C(p+3,3)) complex128 tensor on the GPU; returns beta of the same shape."""
    import numpy as np
    import torch
    R = np.ascontiguousarray(R, np.float64).reshape(-1, 3)
    alpha = alpha.to(torch.complex128).contiguous()
    beta = torch.empty_like(alpha)
    _check(lib().tefmm_sym_m2l(float(k), int(p), R.shape[0], R.ctypes.data, alpha.data_ptr(), beta.data_ptr(),
                               _stream_ptr(stream)))
    return beta


def batch_check(handle, stream=None):
    """Synchronise and raise if the batch's near-field queue had a wait give up
    (tefmm_batch_check)."""
    _check(lib().tefmm_batch_check(handle.h, _stream_ptr(stream)), handle.h)


def _medium(k, d):
    ka = (ctypes.c_double * len(k))(*[float(x) for x in k])
    da = (ctypes.c_double * max(1, len(d)))(*[float(x) for x in d])
    m = MediumC(len(k), da, ka)
    m._keep = (ka, da)
    return m


def default_options(**kw) -> OptionsC:
    o = OptionsC()
    lib().tefmm_default_options(ctypes.byref(o))
    for name, v in kw.items():
        if name == "precision" and isinstance(v, str):
            v = {"fp64": TEFMM_FP64, "fp32": TEFMM_MIXED_FP32, "mixed": TEFMM_MIXED_FP32}[v]
        if name == "normalization" and isinstance(v, str):
            v = {"physical": TEFMM_NORM_PHYSICAL, "paper": TEFMM_NORM_PAPER}[v]
        if name == "sigma_tables" and isinstance(v, str):
            v = SIGMA_TABLES[v]
        setattr(o, name, v)
    return o


def _check(rc, h=None):
    if rc != 0:
        msg = lib().tefmm_last_error(h).decode() if h else ""
        raise TefmmError(rc, msg)


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class TEFMM:
    """Handle of one medium + options.  set_particles(xyz) then evaluate(q)."""

    def __init__(self, k, d, allocator=None, **options):
        """allocator: None (the library's hipMalloc) or "torch" (PyTorch's caching allocator)."""
        self.k, self.d = tuple(k), tuple(d)
        self._med = _medium(self.k, self.d)
        self.opt = default_options(**options)
        h = ctypes.c_void_p()
        _check(lib().tefmm_create(ctypes.byref(h), ctypes.byref(self._med), ctypes.byref(self.opt)))
        self.h = h
        self.n = 0
        self._alloc = None
        if allocator is not None:
            self.set_allocator(allocator)

    def set_allocator(self, allocator):
        """Take the handle's device memory from `allocator` ("torch" or a TorchAllocator;
        None: hipMalloc).  Drops the geometry: call set_particles afterwards."""
        if allocator == "torch":
            allocator = TorchAllocator()
        if allocator is None:
            _check(lib().tefmm_set_allocator(self.h, ALLOC_FN(), FREE_FN(), None), self.h)
        else:
            _check(lib().tefmm_set_allocator(self.h, allocator.alloc, allocator.free, None), self.h)
        self._alloc = allocator

    def close(self):
        if getattr(self, "h", None):
            lib().tefmm_destroy(self.h)  # frees through the allocator, which is still referenced
            self.h = None
            self._alloc = None
            self._xyz = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_surrogate(self, sur):
        """Attach a trained Surrogate (or None); used by the following set_particles calls."""
        self._sur = sur
        _check(lib().tefmm_set_surrogate(self.h, sur.h if sur is not None else None), self.h)

    def set_particles(self, xyz, stream=None):
        """xyz: torch float64 tensor (N, 3) on the GPU (copied to SoA) or numpy (N, 3)."""
        import torch
        if isinstance(xyz, np.ndarray):
            soa = torch.from_numpy(np.ascontiguousarray(np.asarray(xyz, np.float64).T)).cuda()
        else:
            soa = xyz.to(torch.float64).t().contiguous()
        self._xyz = soa
        self.n = soa.shape[1]
        _check(lib().tefmm_set_particles(self.h, self.n, ctypes.c_void_p(soa.data_ptr()), 1, _stream_ptr(stream)),
               self.h)

    def evaluate(self, q, out=None, stream=None):
        """q: torch complex128 on the GPU, shape (N,) or (R, N).  Returns phi, same shape."""
        import torch
        q = q.to(torch.complex128)
        squeeze = q.dim() == 1
        q2 = q.reshape(1, -1) if squeeze else q
        q2 = q2.contiguous()
        R = q2.shape[0]
        if q2.shape[1] != self.n:
            raise ValueError("charge vector length does not match the particles")
        if out is None:
            out = torch.empty_like(q2)
        _check(lib().tefmm_evaluate(self.h, ctypes.c_void_p(q2.data_ptr()), R, ctypes.c_void_p(out.data_ptr()),
                                    _stream_ptr(stream)), self.h)
        return out.reshape(-1) if squeeze else out

    def sigma_derivatives(self, layer, rho, S, method="sommerfeld", stream=None):
        """H_{m,c}(rho_i, S_i) of the layer's Sigma families (tefmm_sigma_derivatives):
        numpy (n, (2p+1)(2p+2)/2) complex128, entry (m + c)(m + c + 1)/2 + m."""
        import numpy as np
        rho = np.ascontiguousarray(rho, np.float64).ravel()
        S = np.ascontiguousarray(S, np.float64).ravel()
        if rho.shape != S.shape:
            raise ValueError("rho and S differ in length")
        P2 = 2 * self.opt.p
        out = np.empty((rho.size, (P2 + 1) * (P2 + 2) // 2), np.complex128)
        m = SIGMA_TABLES[method] if isinstance(method, str) else int(method)
        _check(lib().tefmm_sigma_derivatives(self.h, int(layer), m, rho.size, rho.ctypes.data, S.ctypes.data,
                                              out.ctypes.data, _stream_ptr(stream)), self.h)
        return out

    def delta_derivatives(self, layer, rho, w, method="sommerfeld", stream=None):
        """H_{m,c}(rho_i, w_i) of the layer's Delta family, w = z - z' (tefmm_delta_derivatives):
        numpy (n, (2p+1)(2p+2)/2) complex128, entry (m + c)(m + c + 1)/2 + m."""
        import numpy as np
        rho = np.ascontiguousarray(rho, np.float64).ravel()
        w = np.ascontiguousarray(w, np.float64).ravel()
        if rho.shape != w.shape:
            raise ValueError("rho and w differ in length")
        P2 = 2 * self.opt.p
        out = np.empty((rho.size, (P2 + 1) * (P2 + 2) // 2), np.complex128)
        m = SIGMA_TABLES[method] if isinstance(method, str) else int(method)
        _check(lib().tefmm_delta_derivatives(self.h, int(layer), m, rho.size, rho.ctypes.data, w.ctypes.data,
                                              out.ctypes.data, _stream_ptr(stream)), self.h)
        return out

    def cross_derivatives(self, layer, src_layer, k3, rho, z, zs, stream=None):
        """H_{m,c}(rho_i, z_i, zs_i) of the cross-layer kernel with the source z' derivative of
        order k3 (tefmm_cross_derivatives): numpy (n, (2p+1)(2p+2)/2) complex128."""
        import numpy as np
        rho = np.ascontiguousarray(rho, np.float64).ravel()
        z = np.ascontiguousarray(z, np.float64).ravel()
        zs = np.ascontiguousarray(zs, np.float64).ravel()
        if not (rho.shape == z.shape == zs.shape):
            raise ValueError("rho, z and zs differ in length")
        P2 = 2 * self.opt.p
        out = np.empty((rho.size, (P2 + 1) * (P2 + 2) // 2), np.complex128)
        _check(lib().tefmm_cross_derivatives(self.h, int(layer), int(src_layer), int(k3), rho.size, rho.ctypes.data,
                                              z.ctypes.data, zs.ctypes.data, out.ctypes.data, _stream_ptr(stream)),
               self.h)
        return out

    def gmres(self, b, tau, tol=1e-8, restart=30, max_iter=300, x0=None, stream=None):
        """Solve (I - tau G) x = b by GMRES(restart) through tefmm_gmres (b: torch complex128 on the
        GPU, length N).  Returns (x, info)."""
        import torch
        b = b.to(torch.complex128).contiguous()
        if b.numel() != self.n:
            raise ValueError("right-hand side length does not match the particles")
        x = torch.zeros_like(b) if x0 is None else x0.to(torch.complex128).contiguous().clone()
        info = GmresInfoC()
        tau = complex(tau)
        _check(lib().tefmm_gmres(self.h, tau.real, tau.imag, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                 int(x0 is not None), restart, max_iter, float(tol), _stream_ptr(stream),
                                 ctypes.byref(info)), self.h)
        return x, {f[0]: getattr(info, f[0]) for f in GmresInfoC._fields_}

    def autotune(self, stream=None):
        """Pick tree depth and M2L tile width by timing; returns (depth, targets per workgroup / 16)."""
        d, c = ctypes.c_int(), ctypes.c_int()
        _check(lib().tefmm_autotune(self.h, _stream_ptr(stream), ctypes.byref(d), ctypes.byref(c)), self.h)
        return d.value, c.value

    def reset_timers(self):
        """Start a new averaging window for the phase times reported by stats()."""
        _check(lib().tefmm_reset_timers(self.h), self.h)

    def stats(self) -> dict:
        s = StatsC()
        _check(lib().tefmm_get_stats(self.h, ctypes.byref(s)), self.h)
        d = {f[0]: getattr(s, f[0]) for f in StatsC._fields_}
        d["n_images"] = list(s.n_images)[: s.n_families]
        d["dcim_fit_err"] = list(s.dcim_fit_err)[: s.n_families]
        d["depth"] = list(s.depth)
        return d

    def tree(self, g=0):
        layer, depth, side = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        c = np.zeros(3)
        _check(lib().tefmm_get_tree(self.h, g, ctypes.byref(layer), ctypes.byref(depth),
                                    c.ctypes.data_as(ctypes.c_void_p), ctypes.byref(side)), self.h)
        return {"layer": layer.value, "depth": depth.value, "centre": c, "side": side.value}

    def moments(self, g, level):
        nb = 8 ** level
        nC = (self.opt.p + 1) * (self.opt.p + 2) * (self.opt.p + 3) // 6
        out = np.zeros(nb * nC, np.complex128)
        _check(lib().tefmm_get_moments(self.h, g, level, out.ctypes.data_as(ctypes.c_void_p), 2 * nb * nC), self.h)
        return out.reshape(nb, nC)


def evaluate_batch(handles, qs, outs=None, stream=None, queue=False):
    """Evaluate several TEFMM handles in one graph launch.  qs: list of torch complex128 tensors
    (N_g,) or (R_g, N_g) on the GPU.  Returns the list of outputs (same shapes).  queue: the
    near fields of all geometries in one persistent launch (tefmm_evaluate_batch_queue)."""
    import torch
    n = len(handles)
    qs2, outs2, shapes = [], [], []
    for i, (f, q) in enumerate(zip(handles, qs)):
        q = q.to(torch.complex128)
        shapes.append(q.shape)
        q2 = (q.reshape(1, -1) if q.dim() == 1 else q).contiguous()
        if q2.shape[1] != f.n:
            raise ValueError(f"geometry {i}: charge length does not match")
        qs2.append(q2)
        outs2.append(torch.empty_like(q2) if outs is None else outs[i].reshape(q2.shape))
    H = (ctypes.c_void_p * n)(*[f.h.value for f in handles])
    Q = (ctypes.c_void_p * n)(*[q.data_ptr() for q in qs2])
    P = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs2])
    R = (ctypes.c_int * n)(*[q.shape[0] for q in qs2])
    fn = lib().tefmm_evaluate_batch_queue if queue else lib().tefmm_evaluate_batch
    _check(fn(H, n, Q, R, P, _stream_ptr(stream)), handles[0].h)
    # keep the inputs alive until the caller synchronises (the graph reads them)
    evaluate_batch._keep = (qs2, outs2)
    return [o.reshape(s) for o, s in zip(outs2, shapes)]


def densities(k, d, lp, krho):
    """sigma^{ab}_{m,lp}(krho): array [m][ab][point], ab = uu, ud, du, dd (host FP64)."""
    krho = np.ascontiguousarray(np.asarray(krho, np.complex128).ravel())
    med = _medium(k, d)
    out = np.zeros(len(k) * 4 * len(krho), np.complex128)
    _check(lib().tefmm_densities(ctypes.byref(med), lp, len(krho), krho.ctypes.data_as(ctypes.c_void_p),
                                 out.ctypes.data_as(ctypes.c_void_p)))
    return out.reshape(len(k), 4, len(krho))


def dcim_family(k, d, layer, family, z_lo, z_hi, **options):
    """Complex images (A_j, depth_j) of a same-layer reaction family (host FP64)."""
    med = _medium(k, d)
    opt = default_options(**options)
    cap = 256
    amp = np.zeros(cap, np.complex128)
    dep = np.zeros(cap, np.complex128)
    m = ctypes.c_int()
    fe = ctypes.c_double()
    _check(lib().tefmm_dcim_family(ctypes.byref(med), ctypes.byref(opt), layer, family, float(z_lo), float(z_hi),
                                   cap, ctypes.byref(m), amp.ctypes.data_as(ctypes.c_void_p),
                                   dep.ctypes.data_as(ctypes.c_void_p), ctypes.byref(fe)))
    return amp[: m.value].copy(), dep[: m.value].copy(), fe.value


def dcim_cross(k, d, layer, src_layer, wave, zs, k3p, z_lo, z_hi, **options):
    """Cross-layer complex images (A_j, depth_j) for one source height and z' derivative order."""
    med = _medium(k, d)
    opt = default_options(**options)
    cap = 256
    amp = np.zeros(cap, np.complex128)
    dep = np.zeros(cap, np.complex128)
    m = ctypes.c_int()
    fe = ctypes.c_double()
    _check(lib().tefmm_dcim_cross(ctypes.byref(med), ctypes.byref(opt), layer, src_layer, wave, float(zs), k3p,
                                  float(z_lo), float(z_hi), cap, ctypes.byref(m),
                                  amp.ctypes.data_as(ctypes.c_void_p), dep.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.byref(fe)))
    return amp[: m.value].copy(), dep[: m.value].copy(), fe.value


def taylor_coefficients(x, y, zeta, k, h, order):
    """GPU recurrence: h^{|g|} D^g f / g! ... returned as a_g/h in box units (see tefmm.h)."""
    import torch
    x = torch.as_tensor(np.asarray(x, np.float64)).cuda()
    y = torch.as_tensor(np.asarray(y, np.float64)).cuda()
    z = torch.as_tensor(np.asarray(zeta, np.complex128)).cuda()
    zr = torch.view_as_real(z).contiguous()
    nT = (order + 1) * (order + 2) * (order + 3) // 6
    out = torch.empty(len(x), nT, dtype=torch.complex128, device="cuda")
    _check(lib().tefmm_taylor_coefficients(len(x), ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                           ctypes.c_void_p(zr.data_ptr()), float(k), float(h), order,
                                           ctypes.c_void_p(out.data_ptr())))
    return out.cpu().numpy()


def selftest_mfma() -> int:
    return lib().tefmm_selftest_mfma()


class MLP:
    """The surrogate network through the C ABI (device tensors in, device tensors out)."""

    def __init__(self, n_in, width, n_hidden, n_out, seed=0):
        self.h = ctypes.c_void_p()
        rc = lib().tefmm_mlp_create(ctypes.byref(self.h), n_in, width, n_hidden, n_out, seed)
        if rc != 0:
            raise TefmmError(rc, "mlp_create")
        self.dims = (n_in, width, n_hidden, n_out)

    def _chk(self, rc):
        if rc != 0:
            raise TefmmError(rc, lib().tefmm_mlp_last_error(self.h).decode())

    @property
    def num_params(self):
        return int(lib().tefmm_mlp_num_params(self.h))

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, np.float32)
        assert th.size == self.num_params
        self._chk(lib().tefmm_mlp_set_params(self.h, th.ctypes.data_as(ctypes.c_void_p)))

    def set_split(self, split):
        """Hidden products with BF16 hi + lo operand pairs (tefmm_mlp_set_split)."""
        self._chk(lib().tefmm_mlp_set_split(self.h, int(split)))

    def get_params(self):
        th = np.empty(self.num_params, np.float32)
        self._chk(lib().tefmm_mlp_get_params(self.h, th.ctypes.data_as(ctypes.c_void_p)))
        return th

    def forward(self, x, stream=None):
        import torch
        x = x.contiguous().float()
        y = torch.empty(x.shape[0], self.dims[3], dtype=torch.float32, device=x.device)
        self._chk(lib().tefmm_mlp_forward(self.h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                          ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)))
        return y

    def forward_noalloc(self, x, y, stream=None):
        """tefmm_mlp_forward_noalloc into the caller's y (n x n_out, float32, on the device)."""
        assert x.is_contiguous() and x.dtype == y.dtype and y.is_contiguous()
        assert y.shape == (x.shape[0], self.dims[3])
        self._chk(lib().tefmm_mlp_forward_noalloc(self.h, ctypes.c_void_p(x.data_ptr()), x.shape[0],
                                                  ctypes.c_void_p(y.data_ptr()), _stream_ptr(stream)))
        return y

    def loss_grad(self, x, t, stream=None):
        x = x.contiguous().float()
        t = t.contiguous().float()
        g = np.empty(self.num_params, np.float32)
        L = ctypes.c_double()
        self._chk(lib().tefmm_mlp_loss_grad(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                            x.shape[0], ctypes.byref(L), g.ctypes.data_as(ctypes.c_void_p),
                                            _stream_ptr(stream)))
        return L.value, g

    def adam_step(self, lr, stream=None):
        self._chk(lib().tefmm_mlp_adam_step(self.h, float(lr), _stream_ptr(stream)))

    def train(self, x, t, epochs, batch, lr, seed=0, stream=None):
        x = x.contiguous().float()
        t = t.contiguous().float()
        losses = np.zeros(max(1, epochs))
        self._chk(lib().tefmm_mlp_train(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                        x.shape[0], epochs, batch, float(lr), seed,
                                        losses.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
        return losses[:epochs]

    def close(self):
        if self.h:
            lib().tefmm_mlp_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Surrogate:
    """Trained surrogate for the Sigma tables of one layer (tefmm_surrogate_train)."""

    def __init__(self, k, d, layer, p=8, stream=None, **overrides):
        med = _medium(k, d)
        so = SurOptionsC()
        lib().tefmm_surrogate_default_options(ctypes.byref(med), layer, ctypes.byref(so))
        for name, v in overrides.items():
            setattr(so, name, v)
        opt = default_options(p=p)
        self.h = ctypes.c_void_p()
        rep = SurReportC()
        losses = np.zeros(max(1, so.epochs))
        rc = lib().tefmm_surrogate_train(ctypes.byref(self.h), ctypes.byref(med), ctypes.byref(opt), ctypes.byref(so),
                                         ctypes.byref(rep), losses.ctypes.data_as(ctypes.c_void_p),
                                         _stream_ptr(stream))
        if rc != 0:
            raise TefmmError(rc, "surrogate_train")
        self.options = {f[0]: getattr(so, f[0]) for f in SurOptionsC._fields_}
        self.report = {f[0]: getattr(rep, f[0]) for f in SurReportC._fields_}
        self.losses = losses[: so.epochs]
        self.p = p

    def cell_ok(self, xys):
        xys = np.ascontiguousarray(xys, np.float64).reshape(-1, 3)
        ok = np.zeros(xys.shape[0], np.int32)
        _check(lib().tefmm_surrogate_cell_ok(self.h, xys.shape[0], xys.ctypes.data_as(ctypes.c_void_p),
                                             ok.ctypes.data_as(ctypes.c_void_p)))
        return ok.astype(bool)

    def cell_errors(self):
        o = self.options
        e = np.zeros(o["cells_rho"] * o["cells_s"])
        _check(lib().tefmm_surrogate_cell_errors(self.h, e.ctypes.data_as(ctypes.c_void_p)))
        return e.reshape(o["cells_rho"], o["cells_s"])

    def close(self):
        if self.h:
            lib().tefmm_surrogate_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
