"""ctypes binding of the C ABI in include/kl.h (argument marshalling only).

Every computation runs inside lib/libklmf.so; this module converts Python/PyTorch
arguments to plain pointers and sizes.  Loading fails loudly if the library has not
been built: there is no fallback path.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libklmf.so")

KL_OK, KL_EINVAL, KL_ENOMEM, KL_EHIP, KL_EDOMAIN, KL_ESINGULAR, KL_ENUMERIC, KL_ENOCONV = \
    0, -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "KL_OK", -1: "KL_EINVAL", -2: "KL_ENOMEM", -3: "KL_EHIP", -4: "KL_EDOMAIN",
                -5: "KL_ESINGULAR", -6: "KL_ENUMERIC", -7: "KL_ENOCONV"}
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}
COV_KINDS = {"exp": 0, "sqexp": 1, "exp_l1": 2, "const": 3, "lin": 4}
MAP_KINDS = {"identity": 0, "box": 1, "annulus_nurbs": 2, "annulus_polar": 3, "sine_cube": 4,
             "tensor_nurbs": 5}

# exported symbols declared in include/kl.h
EXPORTS = ["kl_setup", "kl_setup_host", "kl_info", "kl_apply", "kl_apply_noalloc", "kl_stage5", "kl_get_points",
           "kl_get_factor", "kl_kle_field", "kl_eigs", "kl_symeig", "kl_symeig_partial", "kl_symeig_top", "kl_gemm_tall", "kl_gram_tall_workspace", "kl_gram_tall", "kl_profile_enable", "kl_profile_read",
           "kl_stage5_config", "kl_stage5_symmetric", "kl_apply_config", "kl_set_cov", "kl_setup_patches", "kl_patch_count", "kl_patch_info",
           "kl_mlp_create", "kl_mlp_num_params", "kl_mlp_set_params", "kl_mlp_get_params",
           "kl_mlp_forward", "kl_mlp_gradients", "kl_mlp_adam", "kl_mlp_train", "kl_mlp_set_subspace",
           "kl_mlp_destroy",
           "kl_setup_batch", "kl_batch_info", "kl_apply_batch", "kl_batch_config", "kl_eigs_batch",
           "kl_batch_destroy",
           "kl_destroy", "kl_last_error"]


class KLError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_DP3 = ctypes.POINTER(ctypes.c_double) * 3


class KLDesc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("degree", ctypes.c_int32 * 3), ("nelem", ctypes.c_int32 * 3),
                ("knots", _DP3), ("nknots", ctypes.c_int32 * 3),
                ("interp_degree", ctypes.c_int32 * 3), ("interp_nelem", ctypes.c_int32 * 3),
                ("interp_mult", ctypes.c_int32 * 3),
                ("interp_knots", _DP3), ("interp_nknots", ctypes.c_int32 * 3),
                ("map_kind", ctypes.c_int32), ("map_params", ctypes.c_double * 8),
                ("map_degree", ctypes.c_int32 * 3), ("map_knots", _DP3), ("map_nknots", ctypes.c_int32 * 3),
                ("map_ctrl", ctypes.POINTER(ctypes.c_double)), ("map_weights", ctypes.POINTER(ctypes.c_double)),
                ("cov_kind", ctypes.c_int32), ("sigma2", ctypes.c_double),
                ("corr_len", ctypes.c_double * 3)]


class KLEigsOpts(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("block", ctypes.c_int32), ("max_applies", ctypes.c_int32),
                ("tol", ctypes.c_double), ("abs_floor", ctypes.c_double),
                ("precision", ctypes.c_int32), ("refine_fp64", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("guard", ctypes.c_int32), ("max_basis", ctypes.c_int32),
                ("lo_floor", ctypes.c_double), ("coeffs", ctypes.c_int32)]


class KLEigsReport(ctypes.Structure):
    _fields_ = [("n_applies", ctypes.c_int32 * 4), ("n_block_applies", ctypes.c_int32 * 4),
                ("n_restarts", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double), ("t_host_eig", ctypes.c_double),
                ("max_rel_residual", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libklmf.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.kl_setup.argtypes = [ctypes.POINTER(KLDesc), P, ctypes.POINTER(P)]
        L.kl_setup_host.argtypes = [ctypes.POINTER(KLDesc), ctypes.POINTER(P)]
        L.kl_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.kl_apply.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64, P,
                               ctypes.c_int64, P]
        L.kl_stage5.argtypes = L.kl_apply.argtypes
        L.kl_apply_noalloc.argtypes = L.kl_apply.argtypes
        L.kl_get_points.argtypes = [P, P, P]
        L.kl_get_factor.argtypes = [P, ctypes.c_int32, P]
        L.kl_kle_field.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int64, ctypes.c_int32, P,
                                   ctypes.c_int64, P, ctypes.c_int64, P, P]
        L.kl_eigs.argtypes = [P, ctypes.POINTER(KLEigsOpts), P, ctypes.c_int32, P, P,
                              ctypes.c_int64, ctypes.POINTER(KLEigsReport), P]
        L.kl_symeig.argtypes = [ctypes.c_int32, P, P, P]
        L.kl_symeig_partial.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int32]
        L.kl_symeig_top.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, P]
        L.kl_gemm_tall.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64, P,
                                   ctypes.c_int64, ctypes.c_double, ctypes.c_double, P, ctypes.c_int64, P]
        L.kl_gram_tall_workspace.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]
        L.kl_gram_tall_workspace.restype = ctypes.c_int64
        L.kl_gram_tall.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int64, P,
                                   ctypes.c_int64, P, P, ctypes.c_int64, P]
        L.kl_profile_enable.argtypes = [P, ctypes.c_int32]
        L.kl_stage5_config.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P]
        L.kl_stage5_symmetric.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P]
        L.kl_apply_config.argtypes = [P, ctypes.c_int32, P]
        L.kl_profile_read.argtypes = [P, P, P]
        L.kl_set_cov.argtypes = [P, ctypes.c_int32, ctypes.c_double, P]
        L.kl_mlp_create.argtypes = [ctypes.c_int32, P, ctypes.c_uint64, ctypes.POINTER(P)]
        L.kl_mlp_num_params.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
        L.kl_mlp_set_params.argtypes = [P, P]
        L.kl_mlp_get_params.argtypes = [P, P]
        L.kl_mlp_forward.argtypes = [P, ctypes.c_int32, P, P, P]
        L.kl_mlp_gradients.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_double), P, P]
        L.kl_mlp_adam.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, P]
        L.kl_mlp_train.argtypes = [P, ctypes.c_int64, P, P, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_uint64, P, P]
        L.kl_mlp_set_subspace.argtypes = [P, ctypes.c_float]
        L.kl_mlp_destroy.argtypes = [P]
        L.kl_setup_patches.argtypes = [ctypes.c_int32, ctypes.POINTER(KLDesc), P, ctypes.POINTER(P)]
        L.kl_patch_count.argtypes = [P]
        L.kl_patch_info.argtypes = [P, ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int64)] * 4
        L.kl_setup_batch.argtypes = [ctypes.c_int32, ctypes.POINTER(KLDesc), ctypes.POINTER(P)]
        L.kl_batch_info.argtypes = [P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.kl_apply_batch.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P]
        L.kl_batch_config.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
        L.kl_eigs_batch.argtypes = [P, ctypes.POINTER(KLEigsOpts), P, P, P, P]
        L.kl_batch_destroy.argtypes = [P]
        L.kl_destroy.argtypes = [P]
        L.kl_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "kl_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(status):
    if status != KL_OK:
        raise KLError(status, lib().kl_last_error().decode())
    return status


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def grid_to_vec_order(a, d):
    """(m_1, ..., m_d, ...) array -> rows in vec order (first grid index fastest)."""
    a = np.asarray(a, dtype=np.float64)
    axes = list(range(d - 1, -1, -1)) + list(range(d, a.ndim))
    return np.ascontiguousarray(np.transpose(a, axes).reshape((-1,) + a.shape[d:]))


def make_desc(desc):
    """Marshals a workload description dict into the C kl_desc struct.  The host arrays the
    struct points to (knot vectors, control net) are kept alive on the struct (`_keep`)."""
    d = int(desc["dim"])
    c = KLDesc()
    keep = []
    c.dim = d
    deg = list(desc["degree"])
    ne = list(desc.get("nelem") or [0] * d)
    ideg = list(desc.get("interp_degree") or [0] * d)
    ine = list(desc.get("interp_nelem") or [0] * d)
    imu = list(desc.get("interp_mult") or [0] * d)
    for k in range(min(d, 3, len(deg))):
        c.degree[k] = int(deg[k])
        c.nelem[k] = int(ne[k]) if k < len(ne) else 0
        c.interp_degree[k] = int(ideg[k]) if k < len(ideg) else 0
        c.interp_nelem[k] = int(ine[k]) if k < len(ine) else 0
        c.interp_mult[k] = int(imu[k]) if k < len(imu) else 0
    for key, ptrs, lens in (("knots", c.knots, c.nknots), ("interp_knots", c.interp_knots, c.interp_nknots)):
        for k, t in enumerate(desc.get(key) or []):
            if t is None:
                continue
            a = _f64(t)
            keep.append(a)
            ptrs[k] = _dptr(a)
            lens[k] = len(a)
    g = desc["map"]
    c.map_kind = MAP_KINDS[g["kind"]]
    if g["kind"] == "box":
        for k in range(min(d, 3)):
            c.map_params[k] = float(g["lo"][k])
            c.map_params[3 + k] = float(g["hi"][k])
    elif g["kind"] in ("annulus_nurbs", "annulus_polar"):
        c.map_params[0] = float(g.get("r0", 1.0))
        c.map_params[1] = float(g.get("r1", 2.0))
    elif g["kind"] == "sine_cube":
        c.map_params[0] = float(g.get("eps", 0.05))
        amp = list(g.get("amp", [1.0, 0.5, 0.25]))
        for k in range(3):
            c.map_params[1 + k] = float(amp[k]) if k < len(amp) else 0.0
    elif g["kind"] == "tensor_nurbs":
        for k in range(d):
            c.map_degree[k] = int(g["degree"][k])
            a = _f64(g["knots"][k])
            keep.append(a)
            c.map_knots[k] = _dptr(a)
            c.map_nknots[k] = len(a)
        ctrl = grid_to_vec_order(g["ctrl"], d)
        keep.append(ctrl)
        c.map_ctrl = _dptr(ctrl)
        if g.get("weights") is not None:
            w = grid_to_vec_order(g["weights"], d)
            keep.append(w)
            c.map_weights = _dptr(w)
    cov = desc["cov"]
    c.cov_kind = COV_KINDS[cov["kind"]]
    c.sigma2 = float(cov.get("sigma2", 1.0))
    ell = list(cov.get("corr_len", [1.0] * d))
    for k in range(min(d, 3, len(ell))):
        c.corr_len[k] = float(ell[k])
    c._keep = keep
    return c


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Problem:
    """Owns one kl_problem handle (kl_setup / kl_destroy).  `desc` is one description, or
    a list of patch descriptions of one domain (kl_setup_patches)."""

    def __init__(self, desc, host_only=False, stream=None):
        self._h = ctypes.c_void_p()
        self.symmetric = set()          # precisions whose stage 5 is in its symmetric form
        if isinstance(desc, (list, tuple)):
            if host_only:
                raise ValueError("several patches need a GPU (no host-only form)")
            structs = [make_desc(d) for d in desc]     # they keep the host arrays alive
            arr = (KLDesc * len(desc))(*structs)
            check(lib().kl_setup_patches(len(desc), arr, _stream(stream), ctypes.byref(self._h)))
            desc = desc[0]
        else:
            c = make_desc(desc)
            if host_only:
                check(lib().kl_setup_host(ctypes.byref(c), ctypes.byref(self._h)))
            else:
                check(lib().kl_setup(ctypes.byref(c), _stream(stream), ctypes.byref(self._h)))
        N = ctypes.c_int64()
        Nt = ctypes.c_int64()
        n = (ctypes.c_int32 * 3)()
        nt = (ctypes.c_int32 * 3)()
        check(lib().kl_info(self._h, ctypes.byref(N), ctypes.byref(Nt), n, nt))
        self.d = int(desc["dim"])
        self.N, self.Nt = N.value, Nt.value
        self.n = list(n)[:self.d]
        self.nt = list(nt)[:self.d]

    def patches(self):
        """[(N_i, Ntilde_i, dof offset, point offset)] per patch (kl_patch_info)."""
        out = []
        for i in range(int(lib().kl_patch_count(self._h))):
            v = [ctypes.c_int64() for _ in range(4)]
            check(lib().kl_patch_info(self._h, i, *[ctypes.byref(x) for x in v]))
            out.append(tuple(x.value for x in v))
        return out

    def close(self):
        if self._h:
            lib().kl_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def apply(self, x, y, precision="f64", stream=None):
        """y = A~' x for device FP64 tensors of shape (N, nvec), column-major storage
        (a (nvec, N) contiguous tensor viewed transposed, i.e. x.T contiguous)."""
        nvec, ldx, ldy = _colmajor(x, self.N), _ld(x), _ld(y)
        check(lib().kl_apply(self._h, PRECISIONS[precision], nvec, _ptr(x), ldx, _ptr(y), ldy,
                             _stream(stream)))

    def stage5(self, yin, zout, precision="f64", stream=None):
        nvec = _colmajor(yin, self.Nt)
        check(lib().kl_stage5(self._h, PRECISIONS[precision], nvec, _ptr(yin), _ld(yin),
                              _ptr(zout), _ld(zout), _stream(stream)))

    def points(self):
        X = np.zeros((self.Nt, self.d))
        J = np.zeros(self.Nt)
        check(lib().kl_get_points(self._h, ctypes.c_void_p(X.ctypes.data), ctypes.c_void_p(J.ctypes.data)))
        return X, J

    def kle_field(self, lam, evecs, xi=None, variance=True, stream=None):
        """Truncated KL expansion at the Greville points (kl_kle_field).  lam: M host
        eigenvalues; evecs: device (N, M) column-major block (as eigs returns it); xi: device
        (M, m) column-major block of standard-normal draws, or None.  Returns (F, var): device
        tensors of shape (Ntilde, m) (column-major) and (Ntilde,), or None where not asked."""
        import torch
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        M = _colmajor(evecs, self.N)
        if lam.shape != (M,):
            raise ValueError("need one eigenvalue per eigenvector column")
        F = var = None
        m = 0
        if xi is not None:
            m = _colmajor(xi, M)
            F = torch.empty((m, self.Nt), dtype=torch.float64, device=evecs.device).T
        if variance:
            var = torch.empty(self.Nt, dtype=torch.float64, device=evecs.device)
        check(lib().kl_kle_field(self._h, M, ctypes.c_void_p(lam.ctypes.data), _ptr(evecs), _ld(evecs), m,
                                 _ptr(xi) if xi is not None else None, _ld(xi) if xi is not None else 0,
                                 _ptr(F) if F is not None else None, _ld(F) if F is not None else 0,
                                 _ptr(var) if var is not None else None, _stream(stream)))
        return F, var

    def factor(self, k):
        C = np.zeros((self.nt[k], self.n[k]))
        check(lib().kl_get_factor(self._h, k, ctypes.c_void_p(C.ctypes.data)))
        return C

    def set_cov(self, kind, sigma2, corr_len):
        """Replaces the covariance (kind name, variance, per-direction lengths)."""
        ell = (ctypes.c_double * 3)(*([float(v) for v in corr_len] + [1.0] * 3)[:3])
        check(lib().kl_set_cov(self._h, COV_KINDS[kind], float(sigma2), ell))

    def stage5_config(self, precision, rb=0, nsplit=-1):
        """Sets (rb, nsplit; 0/-1 keep) and returns the effective (rb, nsplit)."""
        rbo = ctypes.c_int32()
        nso = ctypes.c_int32()
        check(lib().kl_stage5_config(self._h, PRECISIONS[precision], int(rb), int(nsplit),
                                     ctypes.byref(rbo), ctypes.byref(nso)))
        return rbo.value, nso.value

    def stage5_symmetric(self, on=True, chunk=0, precision="f64"):
        """Symmetric stage 5 on (True) or off for one precision ("f64", "bf16", "bf16x3");
        chunk = row tiles per work item (0 = automatic).  Returns the number of work items
        (0 when off)."""
        out = ctypes.c_int32()
        check(lib().kl_stage5_symmetric(self._h, PRECISIONS[precision], int(bool(on)), int(chunk),
                                        ctypes.byref(out)))
        if on:
            self.symmetric.add(precision)
        else:
            self.symmetric.discard(precision)
        return out.value

    def apply_config(self, fuse_directions=True):
        """Fused (True) or per-direction (False) Kronecker launches; returns whether a
        32-column apply of this problem is fused."""
        out = ctypes.c_int32()
        check(lib().kl_apply_config(self._h, int(bool(fuse_directions)), ctypes.byref(out)))
        return bool(out.value)

    def profile_enable(self, on=True):
        check(lib().kl_profile_enable(self._h, int(bool(on))))

    def profile_read(self):
        """{precision: (timed stage-5 launches, total ms)} since the last enable."""
        cnt = (ctypes.c_int64 * 4)()
        ms = (ctypes.c_double * 4)()
        check(lib().kl_profile_read(self._h, cnt, ms))
        names = {v: k for k, v in PRECISIONS.items()}
        return {names[p]: (int(cnt[p]), float(ms[p])) for p in range(4)}

    def eigs(self, k, precision="f64", block=32, tol=1e-6, abs_floor=1e-12, refine_fp64=True,
             seed=0, x0=None, max_applies=0, guard=0, max_basis=0, lo_floor=0.0, coeffs=False,
             stream=None):
        """k leading eigenpairs; returns (evals numpy, evecs device tensor (N, k) column-major,
        report dict).  coeffs=True returns the B-spline coefficients v = L^{-T} v' instead of
        the standard-form vectors.  The solve is ordered after the work queued on `stream`
        (default: the current stream).  Raises KLError except for KL_ENOCONV, which is
        reported."""
        import torch
        o = KLEigsOpts(k=k, block=block, max_applies=max_applies, tol=tol, abs_floor=abs_floor,
                       precision=PRECISIONS[precision], refine_fp64=int(bool(refine_fp64)),
                       seed=seed, guard=guard, max_basis=max_basis, lo_floor=lo_floor,
                       coeffs=int(bool(coeffs)))
        ev = np.zeros(k)
        V = torch.zeros((k, self.N), dtype=torch.float64, device="cuda").T
        rep = KLEigsReport()
        x0p, n0 = (ctypes.c_void_p(0), 0) if x0 is None else (_ptr(x0), _colmajor(x0, self.N))
        st = lib().kl_eigs(self._h, ctypes.byref(o), x0p, n0, ctypes.c_void_p(ev.ctypes.data),
                           _ptr(V), self.N, ctypes.byref(rep), _stream(stream))
        if st not in (KL_OK, KL_ENOCONV):
            check(st)
        return ev, V, report_dict(rep, st)


class Batch:
    """Owns one kl_batch handle: problems of uneven size applied and solved together.
    Block arenas are CUDA float64 tensors of Ntot * nvec elements; problem i's block is
    the (N_i, nvec) column-major view returned by `block(arena, i, nvec)`."""

    def __init__(self, descs):
        self._h = ctypes.c_void_p()
        structs = [make_desc(d) for d in descs]       # they keep the host arrays alive
        arr = (KLDesc * len(descs))(*structs)
        check(lib().kl_setup_batch(len(descs), arr, ctypes.byref(self._h)))
        self.n = len(descs)
        self.N, self.Nt, self.rowoff = [], [], []
        for i in range(self.n):
            a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
            check(lib().kl_batch_info(self._h, i, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
            self.N.append(a.value)
            self.Nt.append(b.value)
            self.rowoff.append(c.value)
        self.Ntot = sum(self.N)

    def close(self):
        if self._h:
            lib().kl_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def arena(self, nvec):
        import torch
        return torch.zeros(self.Ntot * nvec, dtype=torch.float64, device="cuda")

    def block(self, arena, i, nvec):
        o = nvec * self.rowoff[i]
        return arena[o:o + nvec * self.N[i]].view(nvec, self.N[i]).T

    def apply(self, x, y, nvec, precision="f64", active=None, stream=None):
        act = None if active is None else (ctypes.c_int32 * self.n)(*[int(bool(a)) for a in active])
        check(lib().kl_apply_batch(self._h, PRECISIONS[precision], int(nvec), _ptr(x), _ptr(y),
                                   act, _stream(stream)))

    def config(self, precision, rb=0, lchunk=0):
        """Sets the batched stage-5 tiles; returns (resident workgroups, queue items)."""
        g, it = ctypes.c_int32(), ctypes.c_int32()
        check(lib().kl_batch_config(self._h, PRECISIONS[precision], int(rb), int(lchunk),
                                    ctypes.byref(g), ctypes.byref(it)))
        return g.value, it.value

    def eigs(self, k, precision="f64", block=32, tol=1e-6, abs_floor=1e-12, refine_fp64=True, seed=0,
             max_applies=0, guard=0, max_basis=0, lo_floor=0.0, coeffs=False, stream=None):
        """Returns (evals (n, k) numpy, evecs arena (device), [report dict per problem])."""
        o = KLEigsOpts(k=k, block=block, max_applies=max_applies, tol=tol, abs_floor=abs_floor,
                       precision=PRECISIONS[precision], refine_fp64=int(bool(refine_fp64)),
                       seed=seed, guard=guard, max_basis=max_basis, lo_floor=lo_floor,
                       coeffs=int(bool(coeffs)))
        ev = np.zeros((self.n, k))
        V = self.arena(k)
        reps = (KLEigsReport * self.n)()
        st = lib().kl_eigs_batch(self._h, ctypes.byref(o), ctypes.c_void_p(ev.ctypes.data), _ptr(V), reps,
                                 _stream(stream))
        if st not in (KL_OK, KL_ENOCONV):
            check(st)
        return ev, V, [report_dict(reps[i], st) for i in range(self.n)]


class MLP:
    """Owns one kl_mlp handle: a tanh network sizes[0] -> ... -> sizes[-1] trained on the
    GPU (kl_mlp_*).  Inputs and outputs are row-major FP32 CUDA tensors."""

    def __init__(self, sizes, seed=0):
        self._h = ctypes.c_void_p()
        self.sizes = [int(v) for v in sizes]
        arr = (ctypes.c_int32 * len(self.sizes))(*self.sizes)
        check(lib().kl_mlp_create(len(self.sizes) - 1, arr, int(seed), ctypes.byref(self._h)))
        n = ctypes.c_int64()
        check(lib().kl_mlp_num_params(self._h, ctypes.byref(n)))
        self.n_params = n.value

    def close(self):
        if self._h:
            lib().kl_mlp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        if flat.size != self.n_params:
            raise ValueError("expected %d parameters" % self.n_params)
        check(lib().kl_mlp_set_params(self._h, ctypes.c_void_p(flat.ctypes.data)))

    def get_params(self):
        out = np.zeros(self.n_params, dtype=np.float32)
        check(lib().kl_mlp_get_params(self._h, ctypes.c_void_p(out.ctypes.data)))
        return out

    def forward(self, x, stream=None):
        import torch
        x = _rows_f32(x, self.sizes[0])
        y = torch.empty((x.shape[0], self.sizes[-1]), dtype=torch.float32, device=x.device)
        check(lib().kl_mlp_forward(self._h, x.shape[0], _ptr(x), _ptr(y), _stream(stream)))
        return y

    def gradients(self, x, t, group=0, stream=None):
        """(batch loss, flat device gradients)."""
        import torch
        x = _rows_f32(x, self.sizes[0])
        t = _rows_f32(t, self.sizes[-1])
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double()
        check(lib().kl_mlp_gradients(self._h, x.shape[0], _ptr(x), _ptr(t), int(group), ctypes.byref(loss),
                                     _ptr(g), _stream(stream)))
        return loss.value, g

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        check(lib().kl_mlp_adam(self._h, lr, beta1, beta2, eps, _stream(stream)))

    def set_subspace(self, weight):
        """Weight of the subspace term of the grouped loss (kl_mlp_set_subspace)."""
        check(lib().kl_mlp_set_subspace(self._h, float(weight)))

    def train(self, x, t, group=0, epochs=100, batch=64, lr0=1e-3, lr1=1e-4, seed=0, stream=None):
        """Minibatch Adam training; returns the per-epoch mean loss (numpy)."""
        x = _rows_f32(x, self.sizes[0])
        t = _rows_f32(t, self.sizes[-1])
        if x.shape[0] != t.shape[0]:
            raise ValueError("x and t need the same number of rows")
        losses = np.zeros(int(epochs))
        check(lib().kl_mlp_train(self._h, x.shape[0], _ptr(x), _ptr(t), int(group), int(epochs), int(batch),
                                 float(lr0), float(lr1), int(seed), ctypes.c_void_p(losses.ctypes.data),
                                 _stream(stream)))
        return losses


def _rows_f32(t, width):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or t.dim() != 2 or t.shape[1] != width or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA float32 tensor of shape (rows, %d)" % width)
    return t


def symeig(A):
    """Host dense symmetric eigensolver of the library (w descending, Z columns)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    w = np.zeros(n)
    Z = np.zeros((n, n))          # filled column-major -> read back transposed
    check(lib().kl_symeig(n, ctypes.c_void_p(A.ctypes.data), ctypes.c_void_p(w.ctypes.data),
                          ctypes.c_void_p(Z.ctypes.data)))
    return w, Z.T.copy()


def symeig_partial(A, nv):
    """All eigenvalues (descending) and the eigenvectors of the nv largest."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    w = np.zeros(n)
    Z = np.zeros((max(nv, 1), n))
    check(lib().kl_symeig_partial(n, ctypes.c_void_p(A.ctypes.data), ctypes.c_void_p(w.ctypes.data),
                                  ctypes.c_void_p(Z.ctypes.data), int(nv)))
    return w, Z[:nv].T.copy()


def symeig_top(A, nv):
    """The nv largest eigenvalues (descending) and their eigenvectors."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    w = np.zeros(max(nv, 1))
    Z = np.zeros((max(nv, 1), n))
    check(lib().kl_symeig_top(n, ctypes.c_void_p(A.ctypes.data), int(nv), ctypes.c_void_p(w.ctypes.data),
                              ctypes.c_void_p(Z.ctypes.data)))
    return w[:nv], Z[:nv].T.copy()


def gemm_tall(A, S, out, alpha=1.0, beta=0.0, stream=None):
    """out (N x c) = alpha A S + beta out on the device (kl_gemm_tall): FP64 column-major
    blocks A (N x m), S (m x c) and out (N x c); m = 0 (S with no rows) gives beta out."""
    N, c = int(out.shape[0]), int(out.shape[1])
    m = int(S.shape[0])
    if m and (A.shape[0] != N or A.shape[1] != m or S.shape[1] != c):
        raise ValueError("shapes do not match")
    check(lib().kl_gemm_tall(N, m, c, _ptr(A) if m else None, _ld(A) if m else N, _ptr(S) if m else None,
                             _ld(S) if m else 1, float(alpha), float(beta), _ptr(out), _ld(out), _stream(stream)))
    return out


def gram_tall(A, Bm, stream=None):
    """C = A^T B on the device (kl_gram_tall) for column-major FP64 blocks A (N x m) and
    B (N x c); returns C as a column-major (m, c) device tensor."""
    import torch
    N, m = int(A.shape[0]), int(A.shape[1])
    c = int(Bm.shape[1])
    if Bm.shape[0] != N:
        raise ValueError("A and B need the same number of rows")
    C = torch.empty((c, m), dtype=torch.float64, device=A.device).T
    nw = int(lib().kl_gram_tall_workspace(N, m, c))
    work = torch.empty(max(nw, 1), dtype=torch.float64, device=A.device)
    check(lib().kl_gram_tall(N, m, c, _ptr(A) if m else None, _ld(A) if m else max(N, 1), _ptr(Bm) if c else None,
                             _ld(Bm) if c else max(N, 1), _ptr(C) if m and c else None, _ptr(work), nw,
                             _stream(stream)))
    return C


def report_dict(rep, status=0):
    return {"status": STATUS_NAMES.get(status, status), "n_applies": list(rep.n_applies),
            "n_block_applies": list(rep.n_block_applies), "n_restarts": rep.n_restarts,
            "converged": rep.converged, "t_setup": rep.t_setup, "t_solve": rep.t_solve,
            "t_host_eig": rep.t_host_eig,
            "max_rel_residual": rep.max_rel_residual}


def _colmajor(t, rows):
    """Checks a device FP64 tensor laid out column-major (rows x nvec) and returns nvec."""
    import torch
    if t.dtype != torch.float64 or not t.is_cuda:
        raise ValueError("expected a CUDA float64 tensor")
    if t.dim() == 1:
        t = t[:, None]
    if t.shape[0] != rows or t.stride(0) != 1:
        raise ValueError("expected a column-major (%d, nvec) tensor" % rows)
    return int(t.shape[1])


def _ld(t):
    return int(t.stride(1)) if t.dim() == 2 and t.shape[1] > 1 else int(t.shape[0])
