"""ctypes binding of libdmrg.so (include/dmrg.h).  Argument marshalling only:
every step of sigma, the operator build and Davidson runs in the library.

Device buffers are passed as raw device addresses (e.g. torch.Tensor.data_ptr()
of a CUDA/HIP tensor); host inputs are numpy arrays that the library copies.
"""

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(HERE, "lib", "libdmrg.so")

FP64, FP32, BF16X3 = 0, 1, 2
STATUS = {0: "DMRG_OK", -1: "DMRG_EINVAL", -2: "DMRG_ESHAPE", -3: "DMRG_ENOMEM", -4: "DMRG_EHIP",
          -5: "DMRG_ENOCONV", -6: "DMRG_EINTERNAL"}

EXPORTS = ["dmrg_create", "dmrg_destroy", "dmrg_last_error", "dmrg_build_ops", "dmrg_ops_destroy",
           "dmrg_ops_layout", "dmrg_ops_stats", "dmrg_sigma", "dmrg_diag", "dmrg_diag_noalloc", "dmrg_sigma_batched",
           "dmrg_decimate", "dmrg_decimation_get",
           "dmrg_davidson", "dmrg_davidson_default_opts", "dmrg_profile", "dmrg_mlp_nweights",
           "dmrg_mlp_init", "dmrg_mlp_collect", "dmrg_mlp_train", "dmrg_mlp_apply", "dmrg_autotune",
           "dmrg_launch_shape"]
MLP_NFEAT, MLP_HIDDEN = 18, 256


class Integrals(C.Structure):
    _fields_ = [("K", C.c_int), ("h", C.POINTER(C.c_double)), ("eri", C.POINTER(C.c_double)),
                ("ecore", C.c_double)]


class Mps(C.Structure):
    _fields_ = [("K", C.c_int), ("n_alpha", C.c_int), ("n_beta", C.c_int), ("bond", C.c_int),
                ("nsec", C.POINTER(C.c_int)), ("sec_qn", C.POINTER(C.c_int)),
                ("sec_dim", C.POINTER(C.c_int)), ("blk_off", C.POINTER(C.c_int64)),
                ("data", C.POINTER(C.c_double))]


class BuildOpts(C.Structure):
    _fields_ = [("x_budget_bytes", C.c_size_t), ("t_budget_bytes", C.c_size_t), ("ksplit_tiles", C.c_int64)]


class Stats(C.Structure):
    _fields_ = [("n_psi", C.c_int64), ("n_blocks", C.c_int64), ("n_terms", C.c_int64),
                ("n_rgemm", C.c_int64), ("n_lgemm", C.c_int64), ("flops_sigma", C.c_double),
                ("flops_rstep", C.c_double), ("flops_lstep", C.c_double), ("op_bytes", C.c_double),
                ("build_seconds", C.c_double), ("build_flops", C.c_double),
                ("prof_sigma_calls", C.c_int64), ("prof_launches", C.c_int64),
                ("prof_gemm_ms", C.c_double)]


class DavidsonOpts(C.Structure):
    _fields_ = [("tol_residual", C.c_double), ("max_iter", C.c_int), ("m_max", C.c_int),
                ("precision", C.c_int), ("switch_residual", C.c_double), ("precond", C.c_int),
                ("mlp_weights", C.POINTER(C.c_float)), ("e_ref", C.c_double), ("e_tol", C.c_double),
                ("stop_at_ref", C.c_int), ("stagnation", C.c_int),
                ("trace", C.POINTER(C.c_double)), ("trace_cap", C.c_int), ("precond_shift", C.c_double)]


class DecimationInfo(C.Structure):
    _fields_ = [("nsec", C.c_int), ("kept", C.c_int), ("nblk", C.c_int64), ("ndata", C.c_int64),
                ("discarded", C.c_double), ("entropy", C.c_double)]


class DavidsonStats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("sigma_fp64", C.c_int), ("residual", C.c_double),
                ("seconds", C.c_double), ("seconds_to_ref", C.c_double), ("iters_to_ref", C.c_int),
                ("mlp_fallbacks", C.c_int), ("switch_iter", C.c_int), ("trace_len", C.c_int)]


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def load(path=None):
    path = path or DEFAULT_LIB
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run paper_2311_02854_amd.build.build()")
    lib = C.CDLL(path)
    vp, i64p = C.c_void_p, C.POINTER(C.c_int64)
    lib.dmrg_create.argtypes = [C.POINTER(vp), C.c_int, vp]
    lib.dmrg_destroy.argtypes = [vp]
    lib.dmrg_destroy.restype = None
    lib.dmrg_last_error.argtypes = [vp]
    lib.dmrg_last_error.restype = C.c_char_p
    lib.dmrg_build_ops.argtypes = [vp, C.POINTER(Integrals), C.POINTER(Mps), C.POINTER(BuildOpts), C.POINTER(vp)]
    lib.dmrg_ops_destroy.argtypes = [vp]
    lib.dmrg_ops_destroy.restype = None
    lib.dmrg_ops_layout.argtypes = [vp, i64p, i64p, C.POINTER(C.c_int), i64p]
    lib.dmrg_ops_stats.argtypes = [vp, C.POINTER(Stats)]
    lib.dmrg_sigma.argtypes = [vp, vp, vp, vp, C.c_int]
    lib.dmrg_diag.argtypes = [vp, vp, vp]
    lib.dmrg_diag_noalloc.argtypes = [vp, vp, vp]
    lib.dmrg_decimate.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_double, C.POINTER(DecimationInfo)]
    lib.dmrg_decimation_get.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), i64p, C.POINTER(C.c_double)]
    lib.dmrg_sigma_batched.argtypes = [vp, C.c_int, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.c_int, C.c_int]
    lib.dmrg_autotune.argtypes = [vp, vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.dmrg_launch_shape.argtypes = [vp, C.c_int, C.c_int, C.c_int64]
    lib.dmrg_davidson.argtypes = [vp, vp, vp, C.POINTER(DavidsonOpts), C.POINTER(C.c_double),
                                  C.POINTER(DavidsonStats)]
    lib.dmrg_davidson_default_opts.argtypes = [C.POINTER(DavidsonOpts)]
    lib.dmrg_davidson_default_opts.restype = None
    lib.dmrg_profile.argtypes = [vp, C.c_int]
    fp, dp = C.POINTER(C.c_float), C.POINTER(C.c_double)
    lib.dmrg_mlp_nweights.argtypes = []
    lib.dmrg_mlp_init.argtypes = [fp, C.c_uint64]
    lib.dmrg_mlp_collect.argtypes = [vp, vp, vp, vp, C.c_int, C.c_int, C.c_uint64, C.c_int64, fp, fp, fp, i64p]
    lib.dmrg_mlp_train.argtypes = [vp, C.c_int64, fp, fp, fp, C.c_int, C.c_int, C.c_int, C.c_float, C.c_uint64, fp,
                                   dp, dp]
    lib.dmrg_mlp_apply.argtypes = [vp, vp, fp, vp, vp, C.c_double, vp]
    return lib


class DmrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Context:
    """A library context bound to one device and HIP stream."""

    def __init__(self, device=0, stream=0, lib=None):
        self.lib = lib if lib is not None else load()
        self.h = C.c_void_p()
        self._check(self.lib.dmrg_create(C.byref(self.h), int(device), C.c_void_p(stream or None)))

    def _check(self, rc):
        if rc != 0:
            msg = self.lib.dmrg_last_error(self.h).decode() if self.h else ""
            raise DmrgError(rc, msg)
        return rc

    def close(self):
        if self.h:
            self.lib.dmrg_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_ops(self, ints, mps, x_budget=0, t_budget=0, ksplit_tiles=0):
        """ints: dict(K, h, eri, ecore); mps: synth.SiteMPS (host arrays, copied); budgets in bytes,
        ksplit_tiles the split-k threshold of sigma's L-step (0: library defaults)."""
        h = np.ascontiguousarray(ints["h"], dtype=np.float64)
        eri = np.ascontiguousarray(ints["eri"], dtype=np.float64)
        I = Integrals(int(ints["K"]), _p(h, C.c_double), _p(eri, C.c_double), float(ints.get("ecore", 0.0)))
        nsec, qn, dim, off, data = mps.flat()
        if len(data) == 0:
            data = np.zeros(1)
        if len(off) == 0:
            off = np.zeros(1, np.int64)
        M = Mps(mps.K, mps.Na, mps.Nb, mps.k, _p(nsec, C.c_int), _p(qn, C.c_int), _p(dim, C.c_int),
                _p(off, C.c_int64), _p(data, C.c_double))
        out = C.c_void_p()
        bo = BuildOpts(int(x_budget), int(t_budget), int(ksplit_tiles))
        self._check(self.lib.dmrg_build_ops(self.h, C.byref(I), C.byref(M), C.byref(bo), C.byref(out)))
        return Ops(self, out)


class Ops:
    def __init__(self, ctx, handle):
        self.ctx, self.h = ctx, handle
        n, nb = C.c_int64(), C.c_int64()
        ctx._check(ctx.lib.dmrg_ops_layout(handle, C.byref(n), C.byref(nb), None, None))
        self.n_psi, self.n_blocks = n.value, nb.value
        meta = np.zeros(6 * nb.value, np.int32)
        offs = np.zeros(nb.value, np.int64)
        ctx._check(ctx.lib.dmrg_ops_layout(handle, None, None, _p(meta, C.c_int), _p(offs, C.c_int64)))
        self.blk_meta = meta.reshape(-1, 6)
        self.blk_off = offs

    def destroy(self):
        if self.h:
            self.ctx.lib.dmrg_ops_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def stats(self):
        s = Stats()
        self.ctx._check(self.ctx.lib.dmrg_ops_stats(self.h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}

    def autotune(self, precision=FP64):
        """Pick launch shapes for dmrg_sigma; returns (ms_default, ms_tuned) of one call."""
        a, b = C.c_double(), C.c_double()
        self.ctx._check(self.ctx.lib.dmrg_autotune(self.ctx.h, self.h, int(precision), C.byref(a), C.byref(b)))
        return a.value, b.value

    def launch_shape(self, precision, tile, grid_per_xcd=0):
        """Force the launch shape of dmrg_sigma in one precision (see dmrg.h)."""
        self.ctx._check(self.ctx.lib.dmrg_launch_shape(self.h, int(precision), int(tile), int(grid_per_xcd)))

    def profile(self, enable=True):
        self.ctx._check(self.ctx.lib.dmrg_profile(self.h, int(enable)))

    def sigma(self, psi_ptr, sigma_ptr, precision=FP64):
        self.ctx._check(self.ctx.lib.dmrg_sigma(self.ctx.h, self.h, C.c_void_p(psi_ptr), C.c_void_p(sigma_ptr),
                                                int(precision)))

    def diag(self, out_ptr):
        self.ctx._check(self.ctx.lib.dmrg_diag(self.ctx.h, self.h, C.c_void_p(out_ptr)))

    def decimate(self, psi_ptr, D, direction=0, cutoff=0.0):
        """Keep the D most important states of psi at the bond between the dots.
        Returns dict(sec_qn[nsec, 2], sec_dim[nsec], blk_off[nblk], data[ndata], kept, discarded, entropy)."""
        info = DecimationInfo()
        self.ctx._check(self.ctx.lib.dmrg_decimate(self.ctx.h, self.h, C.c_void_p(psi_ptr), int(D), int(direction),
                                                   float(cutoff), C.byref(info)))
        qn = np.zeros((max(1, info.nsec), 2), np.int32)
        dim = np.zeros(max(1, info.nsec), np.int32)
        off = np.zeros(max(1, info.nblk), np.int64)
        data = np.zeros(max(1, info.ndata), np.float64)
        self.ctx._check(self.ctx.lib.dmrg_decimation_get(self.h, _p(qn, C.c_int), _p(dim, C.c_int),
                                                         _p(off, C.c_int64), _p(data, C.c_double)))
        return {"sec_qn": qn[:info.nsec], "sec_dim": dim[:info.nsec], "blk_off": off[:info.nblk],
                "data": data[:info.ndata], "kept": info.kept, "discarded": info.discarded,
                "entropy": info.entropy}

    def diag_noalloc(self, out_ptr):
        """diag(H) with the library's static scratch instead of allocations."""
        self.ctx._check(self.ctx.lib.dmrg_diag_noalloc(self.ctx.h, self.h, C.c_void_p(out_ptr)))

    def davidson(self, psi_ptr, trace=0, **kw):
        """Lowest eigenpair in place; trace=N also returns the first N per-iteration rows
        (seconds, theta, residual, precision) as out["trace"]."""
        o = DavidsonOpts()
        self.ctx.lib.dmrg_davidson_default_opts(C.byref(o))
        tr = np.zeros((max(1, trace), 4)) if trace else None
        if tr is not None:
            o.trace = _p(tr, C.c_double)
            o.trace_cap = int(trace)
        for k, v in kw.items():
            if k == "mlp_weights":
                o.mlp_weights = v.ctypes.data_as(C.POINTER(C.c_float)) if v is not None else None
                self._mlp_keep = v
            else:
                setattr(o, k, v)
        e = C.c_double()
        st = DavidsonStats()
        rc = self.ctx.lib.dmrg_davidson(self.ctx.h, self.h, C.c_void_p(psi_ptr), C.byref(o), C.byref(e),
                                        C.byref(st))
        if rc not in (0, -5):
            self.ctx._check(rc)
        out = {k: getattr(st, k) for k, _ in DavidsonStats._fields_}
        out["converged"] = rc == 0
        if tr is not None:
            out["trace"] = tr[:st.trace_len].copy()
        return e.value, out


    def mlp_collect(self, psi0_ptr, psi_ref_ptr, max_iter, per_iter, seed, cap):
        """Training pairs of this bond (see dmrg_mlp_collect): (feat[n, NFEAT], dcorr[n], target[n])."""
        feat = np.zeros((cap, MLP_NFEAT), np.float32)
        dc = np.zeros(cap, np.float32)
        tg = np.zeros(cap, np.float32)
        n = C.c_int64()
        self.ctx._check(self.ctx.lib.dmrg_mlp_collect(
            self.ctx.h, self.h, C.c_void_p(psi0_ptr), C.c_void_p(psi_ref_ptr), int(max_iter), int(per_iter),
            int(seed), int(cap), _p(feat, C.c_float), _p(dc, C.c_float), _p(tg, C.c_float), C.byref(n)))
        k = n.value
        return feat[:k], dc[:k], tg[:k]

    def mlp_apply(self, weights, r_ptr, diag_ptr, theta, t_ptr):
        w = np.ascontiguousarray(weights, np.float32)
        self.ctx._check(self.ctx.lib.dmrg_mlp_apply(self.ctx.h, self.h, _p(w, C.c_float), C.c_void_p(r_ptr),
                                                    C.c_void_p(diag_ptr), float(theta), C.c_void_p(t_ptr)))


def mlp_init(lib, seed):
    w = np.zeros(lib.dmrg_mlp_nweights(), np.float32)
    lib.dmrg_mlp_init(_p(w, C.c_float), int(seed))
    return w


def mlp_train(ctx, feat, dcorr, target, weights, epochs=10, batch=4096, lr=1e-3, seed=0, group=0):
    """Train in place on the GPU; returns (loss_before, loss_after).  group > 0 selects the
    per-group direction loss (groups of `group` consecutive pairs)."""
    feat = np.ascontiguousarray(feat, np.float32)
    dcorr = np.ascontiguousarray(dcorr, np.float32)
    target = np.ascontiguousarray(target, np.float32)
    assert weights.dtype == np.float32 and weights.flags.c_contiguous
    lb, la = C.c_double(), C.c_double()
    ctx._check(ctx.lib.dmrg_mlp_train(ctx.h, len(dcorr), _p(feat, C.c_float), _p(dcorr, C.c_float),
                                      _p(target, C.c_float), int(group), int(epochs), int(batch), float(lr),
                                      int(seed), _p(weights, C.c_float), C.byref(lb), C.byref(la)))
    return lb.value, la.value


BATCH_EAGER, BATCH_NO_TUNE = 1, 2


def sigma_batched(ctx, ops_list, psi_ptrs, sigma_ptrs, precision=FP64, flags=0):
    n = len(ops_list)
    arr = C.c_void_p * n
    ctx._check(ctx.lib.dmrg_sigma_batched(ctx.h, n, arr(*[o.h for o in ops_list]), arr(*psi_ptrs),
                                          arr(*sigma_ptrs), int(precision), int(flags)))


def nan():
    return math.nan
