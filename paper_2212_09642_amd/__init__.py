"""Python binding of libvne, the MI355X Lanczos-quadrature engine for the von
Neumann entropy (see include/vne.h for the C ABI it wraps).

Argument marshalling only: every step of the computation runs in the HIP
library.  Host arrays are numpy arrays; device arrays may be passed as torch
tensors (their data_ptr is handed to the library).  Importing the package
does not need a GPU; creating a Context does.  There is no fallback: if
libvne.so is missing the calls raise.
"""
import ctypes
import os

import numpy as np

__all__ = ["VneError", "lib", "version", "laplacian_from_edges", "csr_validate",
           "color_greedy", "Context", "F32", "F64", "MODE_F64", "MODE_DESING",
           "PROBE_RADEMACHER", "PROBE_HUTCHPP", "PROBE_COLORING", "PROBE_DENSE",
           "VALIDATE_SYMMETRIC", "VALIDATE_ZERO_ROWSUM", "LIB_PATH", "EXPORTS", "SELECT_HEURISTIC",
           "SELECT_BOUND", "STOP_BOUND", "STOP_ESTIMATE", "probing_select"]

LIB_PATH = os.environ.get("VNE_LIB_PATH") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                           "libvne.so")

F32, F64 = 0, 1
HOST, DEVICE = 0, 1
MODE_F64, MODE_DESING = 1, 2
PROBE_RADEMACHER, PROBE_HUTCHPP, PROBE_COLORING, PROBE_DENSE = 0, 1, 2, 3
SELECT_HEURISTIC, SELECT_BOUND = 0, 1
STOP_BOUND, STOP_ESTIMATE = 0, 1
VALIDATE_SYMMETRIC, VALIDATE_ZERO_ROWSUM = 1, 2
STATUS = {0: "VNE_OK", -1: "VNE_EINVAL", -2: "VNE_ENOMEM", -3: "VNE_EDEVICE",
          -4: "VNE_ENOTSUP", -5: "VNE_EBUSY", -6: "VNE_ENUMERIC"}

# every symbol include/vne.h declares
EXPORTS = ["vne_version", "vne_laplacian_from_edges", "vne_csr_validate", "vne_color_greedy",
           "vne_ctx_create", "vne_ctx_destroy", "vne_last_error", "vne_ctx_set_stream",
           "vne_ctx_memory", "vne_graph_register", "vne_graph_release", "vne_entropy_estimate",
           "vne_entropy_estimate_batch", "vne_enable_kernel_timing", "vne_kernel_timing",
           "vne_server_start", "vne_server_submit", "vne_server_poll", "vne_server_stats",
           "vne_server_stop", "vne_plan_steps", "vne_plan_probes", "vne_error_bounds",
           "vne_entropy_estimate_adaptive", "vne_entropy_probing", "vne_probing_select", "vne_last_plan",
           "vne_entropy_estimate_noalloc", "vne_rational_quadforms", "vne_hutchpp_adaptive"]


class VneError(RuntimeError):
    def __init__(self, status, msg):
        self.status = status
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("value_dtype", ctypes.c_int32),
                ("location", ctypes.c_int32), ("node_keys", ctypes.c_void_p),
                ("scale", ctypes.c_double)]


class _Probes(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("n_sketch", ctypes.c_int32), ("location", ctypes.c_int32),
                ("colors", ctypes.c_void_p), ("dense", ctypes.c_void_p)]


class _Result(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("quad", ctypes.c_void_p),
                ("alpha", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("k_eff", ctypes.c_void_p), ("norm2", ctypes.c_void_p)]


class _StopRule(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_void_p), ("lam_lo", ctypes.c_double), ("lam_hi", ctypes.c_double),
                ("n_grid", ctypes.c_int32), ("stop", ctypes.c_int32)]


class _RationalCfg(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("poles", ctypes.c_void_p), ("finite_poles", ctypes.c_void_p),
                ("n_finite", ctypes.c_int32), ("ell", ctypes.c_int32), ("c", ctypes.c_double),
                ("cg_tol", ctypes.c_double), ("cg_max", ctypes.c_int32), ("lam_lo", ctypes.c_double),
                ("lam_hi", ctypes.c_double), ("estimate", ctypes.c_int32)]


class _RationalOut(ctypes.Structure):
    _fields_ = [("quad", ctypes.c_void_p), ("psi_steps", ctypes.c_void_p), ("apps_steps", ctypes.c_void_p),
                ("switch_step", ctypes.c_void_p), ("basis", ctypes.c_void_p), ("norm2", ctypes.c_void_p),
                ("err_steps", ctypes.c_void_p), ("cg_iterations", ctypes.c_int64), ("ms", ctypes.c_double)]


HUTCHPP_MAX_ROUNDS = 8


class _HutchppCfg(ctypes.Structure):
    _fields_ = [("rel_eps", ctypes.c_double), ("abs_eps", ctypes.c_double), ("delta", ctypes.c_double),
                ("k_steps", ctypes.c_int32), ("n_pilot", ctypes.c_int32), ("r_first", ctypes.c_int32),
                ("r_max", ctypes.c_int32), ("n_h_max", ctypes.c_int32), ("mode", ctypes.c_uint32),
                ("seed", ctypes.c_uint64)]


class _HutchppResult(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("std_error", ctypes.c_double), ("eps_hat", ctypes.c_double),
                ("n_sketch", ctypes.c_int32), ("n_hutch", ctypes.c_int32), ("capped", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("round_nr", ctypes.c_int32 * HUTCHPP_MAX_ROUNDS),
                ("round_nh", ctypes.c_int32 * HUTCHPP_MAX_ROUNDS),
                ("round_estimate", ctypes.c_double * HUTCHPP_MAX_ROUNDS),
                ("round_sd", ctypes.c_double * HUTCHPP_MAX_ROUNDS), ("krylov_runs", ctypes.c_int64),
                ("ms", ctypes.c_double)]


class _ProbingCfg(ctypes.Structure):
    _fields_ = [("rel_eps", ctypes.c_double), ("select", ctypes.c_int32), ("d_max", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("mode", ctypes.c_uint32), ("lam_lo_fraction", ctypes.c_double),
                ("n_grid", ctypes.c_int32), ("stop", ctypes.c_int32)]


class _ProbingResult(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("d", ctypes.c_int32), ("n_colors", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("capped", ctypes.c_int32), ("unconverged", ctypes.c_int32),
                ("passes", ctypes.c_int32), ("t_pre", ctypes.c_double * 3), ("e1", ctypes.c_double),
                ("q", ctypes.c_double * 2), ("s_lower", ctypes.c_double), ("s_hat", ctypes.c_double),
                ("eps_hat", ctypes.c_double), ("vector_steps", ctypes.c_int64), ("block_steps", ctypes.c_int64),
                ("color_ms", ctypes.c_double), ("lanczos_ms", ctypes.c_double), ("colors", ctypes.c_void_p),
                ("quad", ctypes.c_void_p), ("steps", ctypes.c_void_p), ("quad_cap", ctypes.c_int32)]


class _DistanceChoice(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int32), ("fallback", ctypes.c_int32), ("capped", ctypes.c_int32),
                ("e1", ctypes.c_double), ("q", ctypes.c_double * 2), ("model", ctypes.c_double)]


class _ServerCfg(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("arena_bytes", ctypes.c_uint64), ("max_cols", ctypes.c_int32),
                ("pilot_probes", ctypes.c_int32), ("max_probes", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("z", ctypes.c_double), ("mode", ctypes.c_uint32), ("max_group", ctypes.c_int32),
                ("stop", ctypes.c_int32)]


class _Query(ctypes.Structure):
    _fields_ = [("graph_id", ctypes.c_int32), ("rel_eps", ctypes.c_double), ("m", ctypes.c_int32),
                ("k_steps", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class _QueryResult(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("message", ctypes.c_char * 128), ("estimate", ctypes.c_double),
                ("std_error", ctypes.c_double), ("quad_bound", ctypes.c_double), ("probes", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double)]


class _ServerInfo(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("tasks", ctypes.c_int64), ("queries_done", ctypes.c_int64),
                ("slot_occupancy", ctypes.c_double), ("arena_bytes", ctypes.c_uint64),
                ("arena_in_use", ctypes.c_uint64), ("arena_peak", ctypes.c_uint64), ("active", ctypes.c_int32),
                ("pending", ctypes.c_int32), ("pair_slots", ctypes.c_int64), ("group_tasks", ctypes.c_int64)]


_LIB = None


def lib():
    """Load libvne.so (built in-tree by __graft_entry__.build())."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvne.so not built: run __graft_entry__.build() (%s)" % LIB_PATH)
        # torch first: its HIP runtime is then the one libvne.so binds to, so
        # that the process holds a single runtime (loaded the other way round,
        # two runtimes are mapped and torch's device initialisation fails)
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u64, vp, cp, dbl = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                      ctypes.c_void_p, ctypes.c_char_p, ctypes.c_double)
        P = ctypes.POINTER
        L.vne_version.restype = cp
        L.vne_version.argtypes = []
        L.vne_laplacian_from_edges.restype = i32
        L.vne_laplacian_from_edges.argtypes = [i64, i64, vp, P(i64), P(i64), vp, vp, vp, i32, vp,
                                               P(dbl), cp, i64]
        L.vne_csr_validate.restype = i32
        L.vne_csr_validate.argtypes = [P(_Csr), ctypes.c_uint32, cp, i64]
        L.vne_color_greedy.restype = i32
        L.vne_color_greedy.argtypes = [P(_Csr), i32, vp, P(i32), cp, i64]
        L.vne_ctx_create.restype = i32
        L.vne_ctx_create.argtypes = [ctypes.c_int, u64, vp, P(vp)]
        L.vne_ctx_destroy.restype = None
        L.vne_ctx_destroy.argtypes = [vp]
        L.vne_last_error.restype = cp
        L.vne_last_error.argtypes = [vp]
        L.vne_ctx_set_stream.restype = i32
        L.vne_ctx_set_stream.argtypes = [vp, vp]
        L.vne_ctx_memory.restype = i32
        L.vne_ctx_memory.argtypes = [vp, P(u64)]
        L.vne_graph_register.restype = i32
        L.vne_graph_register.argtypes = [vp, P(_Csr), ctypes.c_uint32, P(i32)]
        L.vne_graph_release.restype = i32
        L.vne_graph_release.argtypes = [vp, i32]
        L.vne_entropy_estimate.restype = i32
        L.vne_entropy_estimate.argtypes = [vp, i32, P(_Probes), i32, ctypes.c_uint32, P(_Result)]
        L.vne_entropy_estimate_batch.restype = i32
        L.vne_entropy_estimate_batch.argtypes = [vp, i32, P(i32), P(_Probes), P(i32), ctypes.c_uint32,
                                                 P(_Result)]
        L.vne_server_start.restype = i32
        L.vne_server_start.argtypes = [vp, P(_ServerCfg), P(vp)]
        L.vne_server_submit.restype = i32
        L.vne_server_submit.argtypes = [vp, P(_Query), P(u64)]
        L.vne_server_poll.restype = i32
        L.vne_server_poll.argtypes = [vp, u64, i32, P(_QueryResult), vp, i32]
        L.vne_server_stats.restype = i32
        L.vne_server_stats.argtypes = [vp, P(_ServerInfo)]
        L.vne_server_stop.restype = i32
        L.vne_server_stop.argtypes = [vp]
        L.vne_error_bounds.restype = i32
        L.vne_error_bounds.argtypes = [vp, i32, i32, vp, vp, vp, vp, i32, dbl, dbl, i32, vp, vp]
        L.vne_plan_steps.restype = i32
        L.vne_entropy_estimate_adaptive.argtypes = [vp, i32, P(_Probes), i32, ctypes.c_uint32, P(_StopRule),
                                                    P(_Result), vp]
        L.vne_entropy_estimate_adaptive.restype = ctypes.c_int
        L.vne_entropy_probing.argtypes = [vp, i32, P(_ProbingCfg), P(_ProbingResult)]
        L.vne_entropy_probing.restype = ctypes.c_int
        L.vne_probing_select.argtypes = [vp, dbl, dbl, dbl, i32, i32, P(_DistanceChoice)]
        L.vne_probing_select.restype = ctypes.c_int
        L.vne_plan_steps.argtypes = [dbl, dbl, dbl, dbl, dbl, i32]
        L.vne_plan_probes.restype = i32
        L.vne_plan_probes.argtypes = [dbl, dbl, dbl, dbl, dbl, i32, i32]
        L.vne_enable_kernel_timing.restype = i32
        L.vne_enable_kernel_timing.argtypes = [vp, i32]
        L.vne_kernel_timing.restype = i32
        L.vne_kernel_timing.argtypes = [vp, i32, P(i64), P(dbl), P(dbl)]
        L.vne_entropy_estimate_noalloc.restype = i32
        L.vne_entropy_estimate_noalloc.argtypes = [vp, i32, P(_Probes), i32, ctypes.c_uint32, P(_Result)]
        L.vne_rational_quadforms.restype = i32
        L.vne_rational_quadforms.argtypes = [vp, i32, P(_Probes), ctypes.c_uint32, P(_RationalCfg), P(_RationalOut)]
        L.vne_hutchpp_adaptive.restype = i32
        L.vne_hutchpp_adaptive.argtypes = [vp, i32, P(_HutchppCfg), P(_HutchppResult), P(dbl), i32]
        L.vne_last_plan.restype = i32
        L.vne_last_plan.argtypes = [vp, P(i32), P(i32)]
        _LIB = L
    return _LIB


def version():
    return lib().vne_version().decode()


def _ptr(a):
    """Address of a numpy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _is_device(a):
    return hasattr(a, "is_cuda") and a.is_cuda


def _check_device(t, dtypes, name):
    """A device tensor handed to the library as a plain pointer must be
    contiguous and of the element type the call reads."""
    if not t.is_contiguous():
        raise ValueError("%s: device tensor must be contiguous" % name)
    if t.dtype not in dtypes:
        raise ValueError("%s: device tensor of dtype %s, expected %s" % (name, t.dtype, " or ".join(map(str, dtypes))))


def _check(st, msg):
    if st != 0:
        raise VneError(st, msg)


def laplacian_from_edges(n_nodes, edges, dtype=np.float32):
    """Laplacian of the largest connected component (eq. (2.3)); see
    vne_laplacian_from_edges.  Returns dict(n, row_ptr, col_idx, values,
    node_ids, scale)."""
    L = lib()
    e = np.ascontiguousarray(np.asarray(edges, np.int64).reshape(-1, 2))
    vd = F64 if np.dtype(dtype) == np.float64 else F32
    n_out, nnz_out, scale = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    msg = ctypes.create_string_buffer(512)
    _check(L.vne_laplacian_from_edges(n_nodes, e.shape[0], _ptr(e), ctypes.byref(n_out),
                                      ctypes.byref(nnz_out), None, None, None, vd, None, None,
                                      msg, 512), msg.value.decode())
    n, nnz = n_out.value, nnz_out.value
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    vals = np.empty(nnz, np.float64 if vd == F64 else np.float32)
    ids = np.empty(n, np.int64)
    _check(L.vne_laplacian_from_edges(n_nodes, e.shape[0], _ptr(e), ctypes.byref(n_out),
                                      ctypes.byref(nnz_out), _ptr(rp), _ptr(ci), _ptr(vals), vd,
                                      _ptr(ids), ctypes.byref(scale), msg, 512), msg.value.decode())
    return dict(n=n, row_ptr=rp, col_idx=ci, values=vals, node_ids=ids, scale=scale.value)


def _csr_struct(row_ptr, col_idx, values, scale, node_keys=None):
    dev = _is_device(row_ptr)
    if not dev:
        row_ptr = np.ascontiguousarray(row_ptr, np.int32)
        col_idx = np.ascontiguousarray(col_idx, np.int32)
        values = np.ascontiguousarray(values)
        if values.dtype not in (np.float32, np.float64):
            values = values.astype(np.float64)
        vd = F64 if values.dtype == np.float64 else F32
    else:
        import torch
        _check_device(row_ptr, (torch.int32,), "row_ptr")
        _check_device(col_idx, (torch.int32,), "col_idx")
        _check_device(values, (torch.float32, torch.float64), "values")
        vd = F64 if values.dtype == torch.float64 else F32
    keys = None
    n = (row_ptr.numel() if dev else row_ptr.size) - 1
    if node_keys is not None:
        keys = np.ascontiguousarray(node_keys, np.int64)
        if keys.size != n:
            raise ValueError("node_keys: %d entries for %d rows" % (keys.size, n))
    nnz = col_idx.numel() if dev else col_idx.size
    s = _Csr(n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(values), vd, DEVICE if dev else HOST,
             _ptr(keys), float(scale))
    return s, (row_ptr, col_idx, values, keys)   # keep arrays alive


def csr_validate(row_ptr, col_idx, values, scale, flags=0):
    s, keep = _csr_struct(row_ptr, col_idx, values, scale)
    msg = ctypes.create_string_buffer(512)
    st = lib().vne_csr_validate(ctypes.byref(s), flags, msg, 512)
    return st, msg.value.decode()


def color_greedy(row_ptr, col_idx, values, d):
    """Greedy distance-d colouring (Algorithm 1); returns (colors int32[n], n_colors)."""
    s, keep = _csr_struct(row_ptr, col_idx, values, 1.0)
    colors = np.empty(s.n, np.int32)
    nc = ctypes.c_int32()
    msg = ctypes.create_string_buffer(512)
    _check(lib().vne_color_greedy(ctypes.byref(s), d, _ptr(colors), ctypes.byref(nc), msg, 512),
           msg.value.decode())
    return colors, nc.value


class Context:
    """A device context (one HIP device, one stream)."""

    def __init__(self, device=0, hbm_budget_bytes=0, stream=None):
        L = lib()
        h = ctypes.c_void_p()
        st = L.vne_ctx_create(device, hbm_budget_bytes, stream, ctypes.byref(h))
        _check(st, L.vne_last_error(None).decode())
        self._h = h
        self._L = L
        self._rows = {}          # graph id -> rows, for the shape checks of probe arrays

    def close(self):
        if getattr(self, "_h", None):
            self._L.vne_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _chk(self, st):
        if st != 0:
            raise VneError(st, self._L.vne_last_error(self._h).decode())

    def set_stream(self, stream):
        self._chk(self._L.vne_ctx_set_stream(self._h, stream))

    def memory(self):
        b = ctypes.c_uint64()
        self._chk(self._L.vne_ctx_memory(self._h, ctypes.byref(b)))
        return b.value

    def register(self, row_ptr, col_idx, values, scale, node_keys=None, validate=0):
        """Register a matrix A = scale * CSR; returns a graph id."""
        s, keep = _csr_struct(row_ptr, col_idx, values, scale, node_keys)
        gid = ctypes.c_int32()
        self._chk(self._L.vne_graph_register(self._h, ctypes.byref(s), validate, ctypes.byref(gid)))
        self._rows[gid.value] = s.n
        return gid.value

    def release(self, gid):
        self._chk(self._L.vne_graph_release(self._h, gid))
        self._rows.pop(gid, None)

    def _check_shapes(self, gid, m, colors, dense):
        """The library reads n colours and an n x m probe block: refuse other
        shapes before it reads past them."""
        n = self._rows.get(gid)
        if n is None:
            return
        if colors is not None and tuple(colors.shape) != (n,):
            raise ValueError("colors: shape %s, expected (%d,)" % (tuple(colors.shape), n))
        if dense is not None and tuple(dense.shape) != (n, m):
            raise ValueError("dense: shape %s, expected (%d, %d)" % (tuple(dense.shape), n, m))

    def estimate(self, gid, kind, m, k, mode, seed=0, n_sketch=0, colors=None, dense=None,
                 want_coeffs=True, _entry="vne_entropy_estimate"):
        """One estimate; returns dict(estimate, quad, alpha, beta, k_eff, norm2)."""
        loc = HOST
        keep = []
        if colors is not None:
            if _is_device(colors):
                import torch
                _check_device(colors, (torch.int32,), "colors")
                loc = DEVICE
            else:
                colors = np.ascontiguousarray(colors, np.int32)
            keep.append(colors)
        if dense is not None:
            if _is_device(dense):
                import torch
                _check_device(dense, (torch.float64 if mode & MODE_F64 else torch.float32,), "dense")
                loc = DEVICE
            else:
                dense = np.ascontiguousarray(dense, np.float64 if mode & MODE_F64 else np.float32)
            keep.append(dense)
        self._check_shapes(gid, m, colors, dense)
        pr = _Probes(kind, m, seed, n_sketch, loc, _ptr(colors), _ptr(dense))
        quad = np.zeros(m)
        kef = np.zeros(m, np.int32)
        nrm = np.zeros(m)
        alpha = np.zeros((m, k)) if want_coeffs else None
        beta = np.zeros((m, k)) if want_coeffs else None
        res = _Result(0.0, _ptr(quad), _ptr(alpha), _ptr(beta), _ptr(kef), _ptr(nrm))
        self._chk(getattr(self._L, _entry)(self._h, gid, ctypes.byref(pr), k, mode, ctypes.byref(res)))
        return dict(estimate=res.estimate, quad=quad, alpha=alpha, beta=beta, k_eff=kef, norm2=nrm)

    def estimate_noalloc(self, gid, kind, m, k, mode, seed=0, colors=None, dense=None, want_coeffs=True):
        """vne_entropy_estimate_noalloc: the estimate of `estimate` with its
        workspace in the library's static scratch array (no allocation)."""
        return self.estimate(gid, kind, m, k, mode, seed=seed, colors=colors, dense=dense,
                             want_coeffs=want_coeffs, _entry="vne_entropy_estimate_noalloc")

    def estimate_batch(self, queries, mode, want_coeffs=False):
        """Several queries in one stacked launch per step.  queries: list of
        dicts with keys gid, kind, m, k and optionally seed, colors, dense
        (host arrays).  Returns one result dict per query."""
        nq = len(queries)
        ids = (ctypes.c_int32 * nq)()
        ks = (ctypes.c_int32 * nq)()
        prs = (_Probes * nq)()
        ress = (_Result * nq)()
        keep, outs = [], []
        vdt = np.float64 if mode & MODE_F64 else np.float32
        for i, q in enumerate(queries):
            m, k = int(q["m"]), int(q["k"])
            colors, dense = q.get("colors"), q.get("dense")
            if colors is not None:
                colors = np.ascontiguousarray(colors, np.int32)
                keep.append(colors)
            if dense is not None:
                dense = np.ascontiguousarray(dense, vdt)
                keep.append(dense)
            self._check_shapes(int(q["gid"]), m, colors, dense)
            ids[i] = int(q["gid"])
            ks[i] = k
            prs[i] = _Probes(int(q["kind"]), m, int(q.get("seed", 0)), 0, HOST, _ptr(colors), _ptr(dense))
            o = dict(quad=np.zeros(m), k_eff=np.zeros(m, np.int32), norm2=np.zeros(m),
                     alpha=np.zeros((m, k)) if want_coeffs else None,
                     beta=np.zeros((m, k)) if want_coeffs else None)
            outs.append(o)
            ress[i] = _Result(0.0, _ptr(o["quad"]), _ptr(o["alpha"]), _ptr(o["beta"]), _ptr(o["k_eff"]),
                              _ptr(o["norm2"]))
        self._chk(self._L.vne_entropy_estimate_batch(self._h, nq, ids, prs, ks, mode, ress))
        for i, o in enumerate(outs):
            o["estimate"] = ress[i].estimate
        return outs

    def error_bounds(self, alpha, beta, k_eff, norm2, steps, lam_lo, lam_hi, n_grid=2000):
        """Theorem 4.8 bracket (lo, hi) per column after min(k_eff, steps) steps."""
        alpha = np.ascontiguousarray(alpha, np.float64)
        beta = np.ascontiguousarray(beta, np.float64)
        k_eff = np.ascontiguousarray(k_eff, np.int32)
        norm2 = np.ascontiguousarray(norm2, np.float64)
        m, k = alpha.shape
        lo = np.zeros(m)
        hi = np.zeros(m)
        self._chk(self._L.vne_error_bounds(self._h, m, k, _ptr(alpha), _ptr(beta), _ptr(k_eff), _ptr(norm2),
                                           int(steps), float(lam_lo), float(lam_hi), int(n_grid), _ptr(lo),
                                           _ptr(hi)))
        return lo, hi

    def estimate_adaptive(self, gid, kind, m, k_max, mode, tol, lam_lo, lam_hi, n_grid=0, seed=0, colors=None,
                          dense=None, want_coeffs=False, stop=STOP_BOUND):
        """Quadratic forms stopped per vector on the Theorem 4.8 upper bound
        (stop=STOP_BOUND) or the eq. (4.10) geometric-mean estimate
        (STOP_ESTIMATE), tolerance tol[c]; returns dict(estimate, quad, steps,
        alpha, beta, k_eff, norm2)."""
        loc = HOST
        keep = []
        if colors is not None:
            if _is_device(colors):
                import torch
                _check_device(colors, (torch.int32,), "colors")
                loc = DEVICE
            else:
                colors = np.ascontiguousarray(colors, np.int32)
            keep.append(colors)
        if dense is not None:
            if _is_device(dense):
                import torch
                _check_device(dense, (torch.float64 if mode & MODE_F64 else torch.float32,), "dense")
                loc = DEVICE
            else:
                dense = np.ascontiguousarray(dense, np.float64 if mode & MODE_F64 else np.float32)
            keep.append(dense)
        tol = np.ascontiguousarray(np.broadcast_to(np.asarray(tol, np.float64), (m,)))
        self._check_shapes(gid, m, colors, dense)
        pr = _Probes(kind, m, seed, 0, loc, _ptr(colors), _ptr(dense))
        rule = _StopRule(_ptr(tol), float(lam_lo), float(lam_hi), int(n_grid), int(stop))
        quad = np.zeros(m)
        steps = np.zeros(m, np.int32)
        kef = np.zeros(m, np.int32)
        nrm = np.zeros(m)
        alpha = np.zeros((m, k_max)) if want_coeffs else None
        beta = np.zeros((m, k_max)) if want_coeffs else None
        res = _Result(0.0, _ptr(quad), _ptr(alpha), _ptr(beta), _ptr(kef), _ptr(nrm))
        self._chk(self._L.vne_entropy_estimate_adaptive(self._h, gid, ctypes.byref(pr), int(k_max), mode,
                                                        ctypes.byref(rule), ctypes.byref(res), _ptr(steps)))
        return dict(estimate=res.estimate, quad=quad, steps=steps, alpha=alpha, beta=beta, k_eff=kef, norm2=nrm)

    def probing(self, gid, rel_eps, select=SELECT_HEURISTIC, d_max=0, k_max=0, mode=MODE_DESING,
                lam_lo_fraction=0.0, n_grid=0, n=None, quad_cap=0, stop=STOP_BOUND):
        """Algorithm 2 (probing with a relative accuracy target).  With n (the
        matrix size) the final colouring is returned; quad_cap > 0 returns the
        first quad_cap psi and stop steps of the final pass.  stop: the
        Krylov stopping rule of step 3 (STOP_BOUND, eq. (4.9); STOP_ESTIMATE,
        eq. (4.10))."""
        cfg = _ProbingCfg(float(rel_eps), int(select), int(d_max), int(k_max), int(mode), float(lam_lo_fraction),
                          int(n_grid), int(stop))
        colors = np.zeros(n, np.int32) if n else None
        quad = np.zeros(quad_cap) if quad_cap > 0 else None
        steps = np.zeros(quad_cap, np.int32) if quad_cap > 0 else None
        r = _ProbingResult()
        r.colors, r.quad, r.steps, r.quad_cap = _ptr(colors), _ptr(quad), _ptr(steps), int(quad_cap)
        self._chk(self._L.vne_entropy_probing(self._h, gid, ctypes.byref(cfg), ctypes.byref(r)))
        out = {f: getattr(r, f) for f, _ in _ProbingResult._fields_ if f not in ("colors", "quad", "steps")}
        out["t_pre"] = list(r.t_pre)
        out["q"] = list(r.q)
        if colors is not None:
            out["colors"] = colors
        if quad is not None:
            w = min(quad_cap, r.n_colors)
            out["quad"], out["steps"] = quad[:w], steps[:w]
        return out

    def enable_kernel_timing(self, on=True):
        self._chk(self._L.vne_enable_kernel_timing(self._h, 1 if on else 0))

    def kernel_timing(self, reset=True):
        n, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        self._chk(self._L.vne_kernel_timing(self._h, 1 if reset else 0, ctypes.byref(n),
                                            ctypes.byref(ms), ctypes.byref(by)))
        return dict(launches=n.value, total_ms=ms.value, bytes=by.value)

    def rational(self, gid, kind, m, mode, steps, poles=None, finite_poles=None, ell=3, c=0.75, cg_tol=0.0,
                 cg_max=0, seed=0, colors=None, dense=None, lam_lo=0.0, lam_hi=0.0, estimate=False):
        """Rational Krylov quadratic forms (vne_rational_quadforms).  poles: the
        pole of each of the steps - 1 steps (np.inf or < 0) for every column,
        or None for the switch rule with finite_poles (its error bound over
        [lam_lo, lam_hi]; estimate: eq. (4.10) instead of the upper bound).
        Returns dict(quad, psi_steps [m, steps], apps_steps [m, steps],
        err_steps [m, steps], switch_step, basis, norm2, cg_iterations, ms)."""
        if colors is not None:
            colors = np.ascontiguousarray(colors, np.int32)
        if dense is not None:
            dense = np.ascontiguousarray(dense, np.float64)
        self._check_shapes(gid, m, colors, dense)
        pl = None if poles is None else np.ascontiguousarray(poles, np.float64)
        if pl is not None and pl.size != steps - 1:
            raise ValueError("poles must have steps - 1 entries")
        fp = None if finite_poles is None else np.ascontiguousarray(finite_poles, np.float64)
        cfg = _RationalCfg(int(steps), _ptr(pl), _ptr(fp), 0 if fp is None else int(fp.size), int(ell), float(c),
                           float(cg_tol), int(cg_max), float(lam_lo), float(lam_hi), 1 if estimate else 0)
        pr = _Probes(kind, m, seed, 0, HOST, _ptr(colors), _ptr(dense))
        quad, nrm = np.zeros(m), np.zeros(m)
        ps, ap, es = np.zeros((m, steps)), np.zeros((m, steps), np.int64), np.zeros((m, steps))
        sw, bs = np.zeros(m, np.int32), np.zeros(m, np.int32)
        o = _RationalOut(_ptr(quad), _ptr(ps), _ptr(ap), _ptr(sw), _ptr(bs), _ptr(nrm), _ptr(es), 0, 0.0)
        self._chk(self._L.vne_rational_quadforms(self._h, gid, ctypes.byref(pr), mode, ctypes.byref(cfg),
                                                 ctypes.byref(o)))
        return dict(quad=quad, psi_steps=ps, apps_steps=ap, err_steps=es, switch_step=sw, basis=bs, norm2=nrm,
                    cg_iterations=o.cg_iterations, ms=o.ms)

    def hutchpp_adaptive(self, gid, k, rel_eps=1e-2, abs_eps=0.0, delta=1e-2, mode=MODE_DESING, seed=0,
                         n_pilot=0, r_first=0, r_max=0, n_h_max=0, quad_cap=0):
        """Adaptive Hutch++ (vne_hutchpp_adaptive): sketch width and Hutchinson
        count picked by the library's rule for P[|err| >= eps_hat] <= delta.
        Returns dict(estimate, std_error, eps_hat, n_sketch, n_hutch, capped,
        rounds=[dict(nr, nh, estimate, sd)], krylov_runs, ms[, quad])."""
        cfg = _HutchppCfg(float(rel_eps), float(abs_eps), float(delta), int(k), int(n_pilot), int(r_first),
                          int(r_max), int(n_h_max), int(mode), int(seed))
        r = _HutchppResult()
        quad = np.zeros(quad_cap) if quad_cap > 0 else None
        self._chk(self._L.vne_hutchpp_adaptive(self._h, gid, ctypes.byref(cfg), ctypes.byref(r),
                                               None if quad is None else quad.ctypes.data_as(
                                                   ctypes.POINTER(ctypes.c_double)), int(quad_cap)))
        out = dict(estimate=r.estimate, std_error=r.std_error, eps_hat=r.eps_hat, n_sketch=r.n_sketch,
                   n_hutch=r.n_hutch, capped=bool(r.capped), krylov_runs=r.krylov_runs, ms=r.ms,
                   rounds=[dict(nr=r.round_nr[i], nh=r.round_nh[i], estimate=r.round_estimate[i],
                                sd=r.round_sd[i]) for i in range(min(r.rounds, HUTCHPP_MAX_ROUNDS))])
        if quad is not None:
            out["quad"] = quad[:min(quad_cap, r.n_sketch + r.n_hutch)]
        return out

    def last_plan(self):
        """Column tile and padded width of the last estimate's Lanczos run."""
        t, mp = ctypes.c_int32(), ctypes.c_int32()
        self._chk(self._L.vne_last_plan(self._h, ctypes.byref(t), ctypes.byref(mp)))
        return dict(tile=t.value, m_pad=mp.value)


def probing_select(T, eps_hat, n, lambda_ub, d_max, use_bound=False):
    """The distance choice of Algorithm 2 (eq. (5.1) fit or Corollary 3.2)."""
    t = None if T is None else np.ascontiguousarray(T, np.float64)
    c = _DistanceChoice()
    st = lib().vne_probing_select(_ptr(t), float(eps_hat), float(n), float(lambda_ub), int(d_max),
                                  1 if use_bound else 0, ctypes.byref(c))
    if st != 0:
        raise VneError(st, "vne_probing_select rejected its arguments")
    return dict(d=c.d, fallback=c.fallback, capped=c.capped, e1=c.e1, q=list(c.q), model=c.model)


def plan_steps(norm2, lambda_max, s_lower, rel_eps, share=0.5, k_max=100):
    """Steps of the serving error rule (Proposition 4.4 with Remark 2.3)."""
    return lib().vne_plan_steps(norm2, lambda_max, s_lower, rel_eps, share, k_max)


def plan_probes(s_hat, sigma, rel_eps, share=0.5, z=2.576, n_min=16, n_max=4096):
    """Probe count of the serving error rule."""
    return lib().vne_plan_probes(s_hat, sigma, rel_eps, share, z, n_min, n_max)


class Server:
    """Serving loop on a context (continuous batching, HBM-budget admission)."""

    def __init__(self, ctx, mode, arena_bytes=0, max_slots=0, max_cols=0, pilot_probes=0, max_probes=0,
                 max_steps=0, z=0.0, max_group=0, stop=0):
        self._ctx = ctx
        self._L = ctx._L
        cfg = _ServerCfg(max_slots, arena_bytes, max_cols, pilot_probes, max_probes, max_steps, z, mode, max_group,
                         stop)
        h = ctypes.c_void_p()
        ctx._chk(self._L.vne_server_start(ctx._h, ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.max_probes = max_probes or 4096

    def submit(self, gid, rel_eps=0.0, m=0, k=0, seed=0):
        t = ctypes.c_uint64()
        q = _Query(gid, rel_eps, m, k, seed)
        self._ctx._chk(self._L.vne_server_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def poll(self, ticket, timeout_ms=-1, want_quad=False):
        """Result dict, or None when not finished within timeout_ms."""
        r = _QueryResult()
        quad = np.zeros(self.max_probes) if want_quad else None
        st = self._L.vne_server_poll(self._h, ticket, timeout_ms, ctypes.byref(r), _ptr(quad),
                                     self.max_probes if want_quad else 0)
        if st == -5:
            return None
        if st != 0:
            raise VneError(st, "poll of ticket %d" % ticket)
        out = dict(status=r.status, message=r.message.decode(), estimate=r.estimate, std_error=r.std_error,
                   quad_bound=r.quad_bound, probes=r.probes, steps=r.steps, queue_ms=r.queue_ms,
                   latency_ms=r.latency_ms)
        if want_quad:
            out["quad"] = quad[:r.probes].copy()
        return out

    def stats(self):
        i = _ServerInfo()
        self._L.vne_server_stats(self._h, ctypes.byref(i))
        return {k: getattr(i, k) for k, _ in _ServerInfo._fields_}

    def stop(self):
        if getattr(self, "_h", None):
            self._L.vne_server_stop(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()
