"""ctypes binding of libmfs_hip.so (the C ABI declared in include/mfs.h).

Argument marshalling only: every step of the method runs in the HIP library.
The functions keep the C names.  Device arrays are torch tensors on the current
HIP device (float64, contiguous); host arrays are numpy arrays.  torch is
imported before the library is loaded so that both use one HIP runtime.
Loading fails loudly when the library has not been built.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfs_hip.so")

MFS_OK, MFS_ERR_ARG, MFS_ERR_GEOMETRY, MFS_ERR_OOM, MFS_ERR_DEVICE, MFS_ERR_STATE, MFS_ERR_NOCONV, MFS_ERR_NUMERIC = range(8)
MFS_RESISTANCE, MFS_MOBILITY = 0, 1
MFS_FP64, MFS_MIXED = 0, 1
PROBLEMS = {"resistance": MFS_RESISTANCE, "mobility": MFS_MOBILITY}
PRECISIONS = {"fp64": MFS_FP64, "mixed": MFS_MIXED}
STATUS_NAMES = {0: "MFS_OK", 1: "MFS_ERR_ARG", 2: "MFS_ERR_GEOMETRY", 3: "MFS_ERR_OOM", 4: "MFS_ERR_DEVICE",
                5: "MFS_ERR_STATE", 6: "MFS_ERR_NOCONV", 7: "MFS_ERR_NUMERIC"}

# Exported symbols, in the order of include/mfs.h.
SYMBOLS = ["mfs_default_params", "mfs_setup", "mfs_precompute_pairs", "mfs_get_pairs", "mfs_get_clusters", "mfs_set_pair_matrices",
           "mfs_get_pair_matrices", "mfs_apply", "mfs_apply_noalloc", "mfs_kernel_sum", "mfs_kernel_sum_work", "mfs_rhs", "mfs_post", "mfs_gmres_solve",
           "mfs_get_sizes", "mfs_destroy", "mfs_last_error", "mfs_server_create", "mfs_server_footprint",
           "mfs_server_submit", "mfs_server_wait", "mfs_server_last_error", "mfs_server_destroy",
           "mfs_keep_fine_factors", "mfs_get_density", "mfs_flow_eval", "mfs_boundary_residual",
           "mfs_setup_ex", "mfs_get_fmm", "mfs_time_kernel_sum"]


class MfsParams(C.Structure):
    _fields_ = [("mu", C.c_double), ("delta_c", C.c_double), ("eps_trunc", C.c_double),
                ("eps_trunc_fine", C.c_double), ("eps_ring", C.c_double), ("n_fp", C.c_int32),
                ("n_ell", C.c_int32), ("m_p", C.c_int32), ("a_ell", C.c_int32), ("gamma", C.c_double),
                ("a_f", C.c_double), ("mobius_r", C.c_double)]


class MfsSolveInfo(C.Structure):
    _fields_ = [("iters_total", C.c_int32), ("outer_steps", C.c_int32), ("rel_resid", C.c_double),
                ("resid_hist", C.POINTER(C.c_double)), ("hist_cap", C.c_int32), ("hist_len", C.c_int32),
                ("ms_rhs", C.c_double), ("ms_iterate", C.c_double), ("ms_post", C.c_double),
                ("n_pairs", C.c_int64), ("matvecs_fp64", C.c_int32), ("matvecs_mixed", C.c_int32),
                ("dense_pairs", C.c_int64), ("direct_pairs", C.c_int64), ("ring_expansions", C.c_int64),
                ("expansion_terms", C.c_int64), ("local_translations", C.c_int64),
                ("local_evaluations", C.c_int64)]


class MfsRequest(C.Structure):
    _fields_ = [("P", C.c_int32), ("centers", C.POINTER(C.c_double)), ("radii", C.POINTER(C.c_double)),
                ("n_src", C.POINTER(C.c_int32)), ("n_col", C.POINTER(C.c_int32)), ("r_src", C.POINTER(C.c_double)),
                ("problem", C.c_int), ("precision", C.c_int), ("given", C.POINTER(C.c_double)),
                ("tol", C.c_double), ("max_iter", C.c_int32)]


class MfsTicketInfo(C.Structure):
    _fields_ = [("ms_queue", C.c_double), ("ms_service", C.c_double), ("ms_total", C.c_double),
                ("ms_precompute", C.c_double), ("footprint_bytes", C.c_int64), ("solve", MfsSolveInfo)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class MfsAllocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class TorchAllocator:
    """Device memory of a context from PyTorch's caching allocator (mfs_setup_ex callbacks).

    Counts calls and live bytes; keep the object alive while the context exists."""

    def __init__(self, stream=None):
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = torch.cuda.current_device()
        self.allocs = self.frees = 0
        self.live = {}

        def _alloc(nbytes, user):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:   # an exception must not cross the C frame: report failure as NULL
                return None
            self.allocs += 1
            self.live[ptr] = int(nbytes)
            return ptr

        def _free(ptr, user):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            finally:
                self.frees += 1
                self.live.pop(ptr, None)

        self._cb = (_ALLOC_FN(_alloc), _FREE_FN(_free))
        self.struct = MfsAllocator(self._cb[0], self._cb[1], None)

    @property
    def live_bytes(self):
        return sum(self.live.values())


_ALLOCATORS = {}   # context handle -> allocator kept alive until mfs_destroy


class MFSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmfs_hip.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2606_11273_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, dp, ip, i64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int64)
    L.mfs_default_params.argtypes = [C.POINTER(MfsParams)]
    L.mfs_default_params.restype = None
    L.mfs_setup.argtypes = [C.POINTER(vp), C.c_int32, dp, dp, ip, ip, dp, C.POINTER(MfsParams), vp]
    L.mfs_setup_ex.argtypes = [C.POINTER(vp), C.c_int32, dp, dp, ip, ip, dp, C.POINTER(MfsParams), vp,
                               C.POINTER(MfsAllocator)]
    L.mfs_precompute_pairs.argtypes = [vp, C.c_int, i64p]
    L.mfs_get_pairs.argtypes = [vp, i64p, ip]
    L.mfs_get_clusters.argtypes = [vp, ip, ip, ip, dp, dp]
    L.mfs_get_fmm.argtypes = [vp, C.c_int, C.c_int, i64p, ip, ip, dp, dp, ip, dp, ip, ip, ip, ip, dp]
    L.mfs_set_pair_matrices.argtypes = [vp, C.c_int, dp, dp]
    L.mfs_get_pair_matrices.argtypes = [vp, C.c_int, dp, dp]
    L.mfs_apply.argtypes = [vp, C.c_int, C.c_int, C.c_int32, vp, vp]
    L.mfs_apply_noalloc.argtypes = [vp, C.c_int, C.c_int, vp, vp]
    L.mfs_kernel_sum.argtypes = [vp, C.c_int, vp, vp, C.c_int32]
    L.mfs_time_kernel_sum.argtypes = [vp, C.c_int, vp, vp, C.c_int32, C.c_int32, dp, dp]
    L.mfs_kernel_sum_work.argtypes = [vp, i64p, C.c_int32]
    L.mfs_rhs.argtypes = [vp, C.c_int, dp, vp]
    L.mfs_post.argtypes = [vp, C.c_int, vp, dp]
    L.mfs_gmres_solve.argtypes = [vp, C.c_int, C.c_int, C.c_int32, dp, dp, vp, C.c_double, C.c_int32,
                                  C.POINTER(MfsSolveInfo)]
    L.mfs_get_sizes.argtypes = [vp, ip, i64p, i64p, i64p]
    L.mfs_keep_fine_factors.argtypes = [vp, C.c_int32]
    L.mfs_get_density.argtypes = [vp, C.c_int32, vp]
    L.mfs_flow_eval.argtypes = [vp, C.c_int, vp, dp, C.c_int64, vp, vp, vp]
    L.mfs_boundary_residual.argtypes = [vp, C.c_int, vp, dp, dp, C.c_int32, vp, dp]
    L.mfs_destroy.argtypes = [vp]
    L.mfs_last_error.argtypes = [vp]
    L.mfs_last_error.restype = C.c_char_p
    L.mfs_server_create.argtypes = [C.POINTER(vp), C.c_size_t, C.c_int32, C.POINTER(MfsParams)]
    L.mfs_server_footprint.argtypes = [vp, C.POINTER(MfsRequest), i64p]
    L.mfs_server_submit.argtypes = [vp, C.POINTER(MfsRequest), i64p]
    L.mfs_server_wait.argtypes = [vp, C.c_int64, dp, C.POINTER(MfsTicketInfo), C.c_int32]
    L.mfs_server_last_error.argtypes = [vp]
    L.mfs_server_last_error.restype = C.c_char_p
    L.mfs_server_destroy.argtypes = [vp]
    for name in SYMBOLS:
        if name not in ("mfs_default_params", "mfs_last_error", "mfs_server_last_error"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _i64p(a):
    return a.ctypes.data_as(C.POINTER(C.c_int64))


def _check(code, ctx):
    if code != MFS_OK:
        msg = lib().mfs_last_error(ctx).decode()
        raise MFSError(code, msg)


def _dev(t, n=None):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError("device arrays must be contiguous float64 torch tensors on the GPU")
    if n is not None and t.numel() < n:
        raise ValueError(f"device array has {t.numel()} entries, need {n}")
    return C.c_void_p(t.data_ptr())


def mfs_default_params():
    p = MfsParams()
    lib().mfs_default_params(C.byref(p))
    return p


def mfs_setup(centers, radii, n_src, n_col, r_src, params=None, stream=None, allocator=None):
    """Returns an opaque context handle (c_void_p).  Host inputs: numpy arrays.  allocator: a
    TorchAllocator (or any object with a .struct MfsAllocator) for mfs_setup_ex, else hipMalloc."""
    centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 2)
    P = centers.shape[0]
    radii = np.ascontiguousarray(np.broadcast_to(radii, (P,)), dtype=np.float64)
    n_src = np.ascontiguousarray(np.broadcast_to(n_src, (P,)), dtype=np.int32)
    n_col = np.ascontiguousarray(np.broadcast_to(n_col, (P,)), dtype=np.int32)
    r_src = np.ascontiguousarray(np.broadcast_to(r_src, (P,)), dtype=np.float64)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    ctx = C.c_void_p()
    if allocator is None:
        code = lib().mfs_setup(C.byref(ctx), P, _dp(centers), _dp(radii), _ip(n_src), _ip(n_col), _dp(r_src),
                               C.byref(params) if params is not None else None, C.c_void_p(stream))
    else:
        code = lib().mfs_setup_ex(C.byref(ctx), P, _dp(centers), _dp(radii), _ip(n_src), _ip(n_col), _dp(r_src),
                                  C.byref(params) if params is not None else None, C.c_void_p(stream),
                                  C.byref(allocator.struct))
    if code != MFS_OK:
        raise MFSError(code, lib().mfs_last_error(None).decode())
    if allocator is not None:
        _ALLOCATORS[ctx.value] = allocator
    return ctx


def mfs_precompute_pairs(ctx, problem):
    n = C.c_int64()
    _check(lib().mfs_precompute_pairs(ctx, PROBLEMS[problem], C.byref(n)), ctx)
    return n.value


def mfs_get_sizes(ctx):
    P, ns, nt, npairs = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().mfs_get_sizes(ctx, C.byref(P), C.byref(ns), C.byref(nt), C.byref(npairs)), ctx)
    return P.value, ns.value, nt.value, npairs.value


def mfs_get_pairs(ctx):
    n = C.c_int64()
    _check(lib().mfs_get_pairs(ctx, C.byref(n), None), ctx)
    out = np.zeros((n.value, 2), dtype=np.int32)
    _check(lib().mfs_get_pairs(ctx, C.byref(n), _ip(out)), ctx)
    return out


def mfs_get_clusters(ctx):
    """The kernel sums' disk order (slots) and the clusters of the two-level sum at arbitrary
    points: dict of slot_body (P), cl_start
    (n_clusters + 1), centre (n_clusters x 2) and radius (n_clusters)."""
    n = C.c_int32()
    _check(lib().mfs_get_clusters(ctx, C.byref(n), None, None, None, None), ctx)
    P = mfs_get_sizes(ctx)[0]
    slot_body = np.zeros(P, dtype=np.int32)
    cl_start = np.zeros(n.value + 1, dtype=np.int32)
    centre = np.zeros((n.value, 2))
    radius = np.zeros(n.value)
    _check(lib().mfs_get_clusters(ctx, C.byref(n), _ip(slot_body), _ip(cl_start), _dp(centre), _dp(radius)), ctx)
    return dict(slot_body=slot_body, cl_start=cl_start, centre=centre, radius=radius)


def mfs_get_fmm(ctx, problem, precision):
    """The hierarchical kernel sum's cells, waves and per-wave lists (mfs_get_fmm): dict of
    cell_lo, cell_hi, cell_c (ncell x 2), cell_r, wave_start (nwave + 1), wave_c (nwave x 2),
    m2l_off, m2l, near_off, near, tier_d2 (P x 3, slot order)."""
    sz = np.zeros(4, dtype=np.int64)
    nul = [None] * 11
    _check(lib().mfs_get_fmm(ctx, PROBLEMS[problem], PRECISIONS[precision], _i64p(sz), *nul), ctx)
    ncell, nwave, nm, nn = (int(v) for v in sz)
    P = mfs_get_sizes(ctx)[0]
    d = dict(cell_lo=np.zeros(ncell, np.int32), cell_hi=np.zeros(ncell, np.int32), cell_c=np.zeros((ncell, 2)),
             cell_r=np.zeros(ncell), wave_start=np.zeros(nwave + 1, np.int32), wave_c=np.zeros((nwave, 2)),
             m2l_off=np.zeros(nwave + 1, np.int32), m2l=np.zeros(max(nm, 1), np.int32),
             near_off=np.zeros(nwave + 1, np.int32), near=np.zeros(max(nn, 1), np.int32), tier_d2=np.zeros((P, 3)))
    _check(lib().mfs_get_fmm(ctx, PROBLEMS[problem], PRECISIONS[precision], _i64p(sz), _ip(d["cell_lo"]),
                             _ip(d["cell_hi"]), _dp(d["cell_c"]), _dp(d["cell_r"]), _ip(d["wave_start"]),
                             _dp(d["wave_c"]), _ip(d["m2l_off"]), _ip(d["m2l"]), _ip(d["near_off"]), _ip(d["near"]),
                             _dp(d["tier_d2"])), ctx)
    d["m2l"], d["near"] = d["m2l"][:nm], d["near"][:nn]
    return d


def _pair_sizes(ctx, n_src):
    pr = mfs_get_pairs(ctx)
    n = 2 * (n_src[pr[:, 0]] + n_src[pr[:, 1]]) if len(pr) else np.zeros(0, dtype=np.int64)
    return pr, n.astype(np.int64)


def mfs_set_pair_matrices(ctx, problem, A_list, E_list):
    A = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in A_list]) if A_list
                             else np.zeros(1))
    E = np.ascontiguousarray(np.concatenate([np.asarray(e, dtype=np.float64).ravel() for e in E_list]) if E_list
                             else np.zeros(1))
    _check(lib().mfs_set_pair_matrices(ctx, PROBLEMS[problem], _dp(A), _dp(E)), ctx)


def mfs_get_pair_matrices(ctx, problem, n_src):
    pr, n = _pair_sizes(ctx, np.asarray(n_src))
    A = np.zeros(max(1, int(np.sum(n * n))))
    E = np.zeros(max(1, int(np.sum(6 * n))))
    _check(lib().mfs_get_pair_matrices(ctx, PROBLEMS[problem], _dp(A), _dp(E)), ctx)
    As, Es, ao, eo = [], [], 0, 0
    for m in n:
        As.append(A[ao:ao + m * m].reshape(m, m))
        Es.append(E[eo:eo + 6 * m].reshape(6, m))
        ao += m * m
        eo += 6 * m
    return As, Es


def mfs_apply(ctx, problem, precision, mu, u, n_rhs=1):
    _check(lib().mfs_apply(ctx, PROBLEMS[problem], PRECISIONS[precision], n_rhs, _dev(mu), _dev(u)), ctx)


def mfs_apply_noalloc(ctx, problem, precision, mu, u):
    """mfs_apply for one vector with no device allocation (split partials in the static scratch)."""
    _check(lib().mfs_apply_noalloc(ctx, PROBLEMS[problem], PRECISIONS[precision], _dev(mu), _dev(u)), ctx)


def mfs_kernel_sum_work(ctx, reset=False):
    """(direct pairs, disk expansions, cluster expansions, local translations, local evaluations)
    counted by the kernel sums since setup or the last reset."""
    w = np.zeros(5, dtype=np.int64)
    _check(lib().mfs_kernel_sum_work(ctx, w.ctypes.data_as(C.POINTER(C.c_int64)), int(bool(reset))), ctx)
    return tuple(int(v) for v in w)


def mfs_kernel_sum(ctx, precision, sigma, u, skip=1):
    """skip: 0 all sources, 1 skip the target's own disk, 2 also skip its contact partners."""
    _check(lib().mfs_kernel_sum(ctx, PRECISIONS[precision], _dev(sigma), _dev(u), int(skip)), ctx)


def mfs_time_kernel_sum(ctx, precision, sigma, u, skip=2, reps=5):
    """(ms to pack and form the records, average ms of one sum launch), HIP events on the
    context's stream."""
    a, b = C.c_double(), C.c_double()
    _check(lib().mfs_time_kernel_sum(ctx, PRECISIONS[precision], _dev(sigma), _dev(u), int(skip), int(reps),
                                     C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def mfs_rhs(ctx, problem, given, b):
    given = np.ascontiguousarray(given, dtype=np.float64)
    _check(lib().mfs_rhs(ctx, PROBLEMS[problem], _dp(given), _dev(b)), ctx)


def mfs_keep_fine_factors(ctx, keep=True):
    _check(lib().mfs_keep_fine_factors(ctx, int(bool(keep))), ctx)


def mfs_get_density(ctx, rhs, mu):
    _check(lib().mfs_get_density(ctx, int(rhs), _dev(mu)), ctx)


def _dev_i32(t):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
        raise TypeError("body indices must be a contiguous int32 torch tensor on the GPU")
    return C.c_void_p(t.data_ptr())


def mfs_flow_eval(ctx, problem, mu, given, pts, body, u):
    """pts (device float64, 2 n), body (device int32, n; -1 fluid), u (device float64, 2 n)."""
    n = body.numel()
    g = None if given is None else np.ascontiguousarray(given, dtype=np.float64)
    _check(lib().mfs_flow_eval(ctx, PROBLEMS[problem], _dev(mu), None if g is None else _dp(g), n,
                               _dev(pts, 2 * n), _dev_i32(body), _dev(u, 2 * n)), ctx)


def mfs_boundary_residual(ctx, problem, mu, given, rigid, n_per_body, eps=None):
    """Returns eps_max; eps (device float64, P n_per_body) receives the pointwise residuals."""
    g = None if given is None else np.ascontiguousarray(given, dtype=np.float64)
    rig = np.ascontiguousarray(rigid, dtype=np.float64)
    P = rig.size // 3
    out = C.c_double(0.0)
    if eps is not None:
        _dev(eps, P * int(n_per_body))
    _check(lib().mfs_boundary_residual(ctx, PROBLEMS[problem], _dev(mu), None if g is None else _dp(g), _dp(rig),
                                       int(n_per_body), None if eps is None else _dev(eps), C.byref(out)), ctx)
    return out.value


def mfs_post(ctx, problem, mu, P):
    out = np.zeros((P, 3))
    _check(lib().mfs_post(ctx, PROBLEMS[problem], _dev(mu), _dp(out)), ctx)
    return out


def mfs_gmres_solve(ctx, problem, precision, rhs, tol, max_iter=500, x0=None, hist_cap=1000, allow_noconv=False):
    """rhs: (P,3) or (n_rhs,P,3) host array.  Returns (out, info dict)."""
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    n_rhs = 1 if rhs.ndim == 2 else rhs.shape[0]
    out = np.zeros_like(rhs)
    hist = np.zeros(hist_cap)
    info = MfsSolveInfo()
    info.resid_hist = _dp(hist)
    info.hist_cap = hist_cap
    code = lib().mfs_gmres_solve(ctx, PROBLEMS[problem], PRECISIONS[precision], n_rhs, _dp(rhs), _dp(out),
                                 _dev(x0) if x0 is not None else None, tol, max_iter, C.byref(info))
    if not (code == MFS_OK or (allow_noconv and code == MFS_ERR_NOCONV)):
        _check(code, ctx)
    d = dict(iters=info.iters_total, outer=info.outer_steps, rel_resid=info.rel_resid,
             hist=hist[:info.hist_len].copy(), ms_rhs=info.ms_rhs, ms_iterate=info.ms_iterate, ms_post=info.ms_post,
             n_pairs=info.n_pairs, matvecs_fp64=info.matvecs_fp64, matvecs_mixed=info.matvecs_mixed,
             dense_pairs=info.dense_pairs, direct_pairs=info.direct_pairs, ring_expansions=info.ring_expansions,
             expansion_terms=info.expansion_terms, local_translations=info.local_translations,
             local_evaluations=info.local_evaluations, status=STATUS_NAMES[code])
    return out, d


def mfs_destroy(ctx):
    if ctx:
        lib().mfs_destroy(ctx)
        _ALLOCATORS.pop(ctx.value, None)


# -- serving ----------------------------------------------------------------------------

def mfs_server_create(hbm_budget_bytes=0, max_slots=4, params=None):
    srv = C.c_void_p()
    code = lib().mfs_server_create(C.byref(srv), int(hbm_budget_bytes), int(max_slots),
                                   C.byref(params) if params is not None else None)
    if code != MFS_OK:
        raise MFSError(code, "server creation failed")
    return srv


def _request(centers, radii, n_src, n_col, r_src, problem, precision, given, tol, max_iter):
    """Build an MfsRequest; returns (request, keep-alive arrays)."""
    centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 2)
    P = centers.shape[0]
    arrs = dict(centers=centers,
                radii=np.ascontiguousarray(np.broadcast_to(radii, (P,)), dtype=np.float64),
                n_src=np.ascontiguousarray(np.broadcast_to(n_src, (P,)), dtype=np.int32),
                n_col=np.ascontiguousarray(np.broadcast_to(n_col, (P,)), dtype=np.int32),
                r_src=np.ascontiguousarray(np.broadcast_to(r_src, (P,)), dtype=np.float64),
                given=np.ascontiguousarray(given, dtype=np.float64).reshape(P, 3))
    r = MfsRequest(P, _dp(arrs["centers"]), _dp(arrs["radii"]), _ip(arrs["n_src"]), _ip(arrs["n_col"]),
                   _dp(arrs["r_src"]), PROBLEMS[problem], PRECISIONS[precision], _dp(arrs["given"]), float(tol),
                   int(max_iter))
    return r, arrs


def _srv_check(code, srv):
    if code != MFS_OK:
        raise MFSError(code, lib().mfs_server_last_error(srv).decode())


def mfs_server_footprint(srv, centers, radii, n_src, n_col, r_src, problem, precision, given, tol, max_iter=300):
    r, keep = _request(centers, radii, n_src, n_col, r_src, problem, precision, given, tol, max_iter)
    b = C.c_int64()
    _srv_check(lib().mfs_server_footprint(srv, C.byref(r), C.byref(b)), srv)
    return b.value


def mfs_server_submit(srv, centers, radii, n_src, n_col, r_src, problem, precision, given, tol, max_iter=300):
    """Queue one solve; returns its ticket."""
    r, keep = _request(centers, radii, n_src, n_col, r_src, problem, precision, given, tol, max_iter)
    t = C.c_int64()
    _srv_check(lib().mfs_server_submit(srv, C.byref(r), C.byref(t)), srv)
    return t.value


def mfs_server_wait(srv, ticket, P, timeout_ms=-1, allow_noconv=False):
    """Wait for a ticket; returns (out (P, 3), dict of timings and solve figures)."""
    out = np.zeros((P, 3))
    info = MfsTicketInfo()
    code = lib().mfs_server_wait(srv, int(ticket), _dp(out), C.byref(info), int(timeout_ms))
    if code != MFS_OK and not (allow_noconv and code == MFS_ERR_NOCONV):
        _srv_check(code, srv)
    s = info.solve
    return out, dict(ms_queue=info.ms_queue, ms_service=info.ms_service, ms_total=info.ms_total,
                     ms_precompute=info.ms_precompute, footprint=info.footprint_bytes, iters=s.iters_total,
                     outer=s.outer_steps, rel_resid=s.rel_resid, n_pairs=s.n_pairs, dense_pairs=s.dense_pairs,
                     direct_pairs=s.direct_pairs,
                     status=code)


def mfs_server_destroy(srv):
    lib().mfs_server_destroy(srv)
