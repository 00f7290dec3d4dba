"""Thin ctypes binding of libbbp (include/bbp.h): argument marshalling only.

Every computation runs in the HIP library; this module converts NumPy arrays
to pointers, raises on error status, and unpacks message buffers.  The library
must be built (``python -m paper_2301_05844_amd.build``); importing this module
without it raises ``ImportError``.
"""

import ctypes
import os

import numpy as np

try:
    # torch (device memory, streams) ships its own HIP runtime; loading it
    # before libbbp makes the library bind to that same runtime, so one HIP
    # runtime serves both in this process.
    import torch  # noqa: F401
except ImportError:
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbbp.so")

EXPORTS = (
    "bbp_create", "bbp_set_option", "bbp_set_stream", "bbp_set_allocator",
    "bbp_set_tensors", "bbp_get_tensors",
    "bbp_sweep", "bbp_expect_site", "bbp_expect_bond", "bbp_expect_sites",
    "bbp_expect_bonds", "bbp_expect_terms", "bbp_rdm_sites", "bbp_rdm_bonds", "bbp_trace_distance",
    "bbp_log_norm", "bbp_get_messages",
    "bbp_set_messages", "bbp_stats", "bbp_kernel_stats",
    "bbp_kernel_stats_padded", "bbp_kernel_stats_reset", "bbp_memory", "bbp_last_error", "bbp_destroy",
    "bbp_server_estimate", "bbp_server_create", "bbp_server_submit",
    "bbp_server_poll", "bbp_server_cancel", "bbp_server_stats",
    "bbp_server_sweeps", "bbp_server_error", "bbp_server_destroy",
    "bbp_update_workspace", "bbp_update_message", "bbp_update_message_noalloc",
    "bbp_update_last_error", "bbp_ite_step", "bbp_ite_fit", "bbp_svd_jacobi",
)

OUT_SZ, OUT_SS, OUT_LOGNORM = 1, 2, 4

# bbp_alloc_fn / bbp_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
REQ_STATES = {0: "queued", 1: "running", 2: "done", 3: "failed", 4: "cancelled"}


class Request(ctypes.Structure):
    """bbp_request of include/bbp.h."""
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("bx", ctypes.c_int32), ("by", ctypes.c_int32),
                ("D", ctypes.c_int32), ("chi", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("outputs", ctypes.c_int32),
                ("n_site_ops", ctypes.c_int32), ("n_bond_ops", ctypes.c_int32),
                ("tol", ctypes.c_double)]

class UpdateSpec(ctypes.Structure):
    """bbp_update_spec of include/bbp.h."""
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("D", ctypes.c_int32), ("d", ctypes.c_int32),
                ("chi", ctypes.c_int32), ("n_fit", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("slot", ctypes.c_uint64)]


STATUS = {0: "BBP_OK", 1: "BBP_EINVAL", 2: "BBP_ENOMEM", 3: "BBP_EDEVICE",
          4: "BBP_ESTATE", 5: "BBP_ENUMERIC"}


class BBPError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libbbp.so not built at {LIB_PATH}; run "
                          "python -m paper_2301_05844_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    c_int, c_double, c_size = ctypes.c_int32, ctypes.c_double, ctypes.c_size_t
    P = ctypes.c_void_p
    dp = ctypes.POINTER(c_double)
    ip = ctypes.POINTER(c_int)
    sig = {
        "bbp_create": [ctypes.POINTER(P)] + [c_int] * 9,
        "bbp_set_option": [P, ctypes.c_char_p, c_double],
        "bbp_set_stream": [P, P],
        "bbp_set_allocator": [P, ALLOC_FN, FREE_FN, P],
        "bbp_set_tensors": [P, dp, c_size],
        "bbp_get_tensors": [P, dp, c_size],
        "bbp_sweep": [P, c_int, dp],
        "bbp_expect_site": [P, c_int, c_int, dp, dp],
        "bbp_expect_bond": [P, c_int, c_int, c_int, c_int, dp, dp],
        "bbp_expect_sites": [P, c_int, ip, ip, dp, dp],
        "bbp_expect_bonds": [P, c_int, ip, ip, ip, ip, dp, dp],
        "bbp_expect_terms": [P, c_int, ip, ip, dp, c_int, ip, ip, ip, ip, dp, dp, dp],
        "bbp_rdm_sites": [P, c_int, ip, ip, dp],
        "bbp_rdm_bonds": [P, c_int, ip, ip, ip, ip, dp],
        "bbp_trace_distance": [c_int, dp, dp, dp],
        "bbp_svd_jacobi": [c_int, c_int, c_int, c_int, P, P, P, P, P, P, c_int, c_double, P],
        "bbp_ite_step": [P, dp, c_int, dp],
        "bbp_ite_fit": [c_int, c_int, c_int, c_int, dp, dp, dp, c_int, dp, dp, dp],
        "bbp_log_norm": [P, dp, ip],
        "bbp_get_messages": [P, dp, c_size, ctypes.POINTER(c_size)],
        "bbp_set_messages": [P, dp, c_size],
        "bbp_stats": [P, ip, dp],
        "bbp_kernel_stats": [P, c_int, ctypes.POINTER(ctypes.c_char_p),
                             ctypes.POINTER(ctypes.c_int64), dp, dp, dp],
        "bbp_kernel_stats_padded": [P, c_int, dp, dp],
        "bbp_kernel_stats_reset": [P],
        "bbp_memory": [P, ctypes.POINTER(c_size), ctypes.POINTER(c_size)],
        "bbp_server_estimate": [ctypes.POINTER(Request), ctypes.POINTER(c_size)],
        "bbp_server_create": [ctypes.POINTER(P), c_size, c_int],
        "bbp_server_submit": [P, ctypes.POINTER(Request), dp, c_size, dp,
                              ctypes.POINTER(ctypes.c_int64)],
        "bbp_server_poll": [P, ctypes.c_int64, ip, dp, c_size,
                            ctypes.POINTER(c_size), dp],
        "bbp_server_cancel": [P, ctypes.c_int64],
        "bbp_server_stats": [P, ip, ip, ctypes.POINTER(c_size), ip],
        "bbp_server_sweeps": [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                              ip, dp],
        "bbp_update_workspace": [ctypes.POINTER(UpdateSpec), ctypes.POINTER(c_size)],
        "bbp_update_message": [ctypes.POINTER(UpdateSpec), P, P, ip, P, ip, P, ip, P, ip,
                               dp, P],
        "bbp_update_message_noalloc": [ctypes.POINTER(UpdateSpec), P, P, ip, P, ip, P, ip,
                                       P, ip, dp, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.bbp_last_error.argtypes = [P]
    lib.bbp_last_error.restype = ctypes.c_char_p
    lib.bbp_destroy.argtypes = [P]
    lib.bbp_destroy.restype = None
    lib.bbp_server_error.argtypes = [P, ctypes.c_int64]
    lib.bbp_server_error.restype = ctypes.c_char_p
    lib.bbp_server_destroy.argtypes = [P]
    lib.bbp_server_destroy.restype = None
    lib.bbp_update_last_error.argtypes = []
    lib.bbp_update_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


class BlockBP:
    """One libbbp context.  ``finite``: ``BlockBP(Lx=, Ly=, bx=, by=, D=,
    chi=)``; infinite: ``BlockBP(infinite=True, ucx=, ucy=, bx=, by=, D=,
    chi=)``.  Options (``chi_env``, ``n_fit``, ``seed``, ``d``) are passed to
    ``bbp_set_option`` before the tensors."""

    def __init__(self, D, chi, bx, by, Lx=0, Ly=0, infinite=False, ucx=0,
                 ucy=0, stream=None, allocator=None, **options):
        self._ctx = ctypes.c_void_p()
        self._alloc_cb = None
        st = _lib.bbp_create(ctypes.byref(self._ctx), int(bool(infinite)),
                             Lx, Ly, ucx, ucy, bx, by, D, chi)
        if st != 0:
            raise BBPError(st, "bbp_create rejected its arguments")
        self.D, self.chi = D, chi
        self.d = int(options.get("d", 2))
        for k, v in options.items():
            self._check(_lib.bbp_set_option(self._ctx, k.encode(), float(v)))
        if stream is not None:
            self.set_stream(stream)
        if allocator is not None:
            self.set_allocator(*allocator)

    def _check(self, st):
        if st != 0:
            raise BBPError(st, _lib.bbp_last_error(self._ctx).decode())

    def set_stream(self, stream):
        """``stream``: a torch.cuda.Stream, an integer handle, or None."""
        handle = getattr(stream, "cuda_stream", stream)
        self._check(_lib.bbp_set_stream(self._ctx, ctypes.c_void_p(handle)))

    def set_allocator(self, alloc, free):
        """Device memory through ``alloc(nbytes) -> int`` (0 on failure) and
        ``free(ptr)`` (bbp_set_allocator); ``None, None`` restores
        hipMalloc/hipFree.  Before ``set_tensors``."""
        if alloc is None and free is None:
            cbs = (ALLOC_FN(), FREE_FN())
        else:
            def _a(nbytes, _user):
                try:
                    return int(alloc(int(nbytes))) or None
                except Exception:  # reported to the library as out of memory
                    return None

            def _f(ptr, _user):
                free(int(ptr))
            cbs = (ALLOC_FN(_a), FREE_FN(_f))
        self._check(_lib.bbp_set_allocator(self._ctx, cbs[0], cbs[1], None))
        self._alloc_cb = cbs  # kept alive while the context may call them

    def set_option(self, key, value):
        self._check(_lib.bbp_set_option(self._ctx, key.encode(), float(value)))

    def set_tensors(self, A):
        A = np.ascontiguousarray(A, dtype=np.float64)
        self._check(_lib.bbp_set_tensors(self._ctx, _dptr(A), A.size))
        self._tensor_shape = A.shape

    def get_tensors(self):
        """bbp_get_tensors: the site tensors, shape as last set."""
        out = np.zeros(self._tensor_shape)
        self._check(_lib.bbp_get_tensors(self._ctx, _dptr(out), out.size))
        return out

    def sweep(self, n=1):
        r = ctypes.c_double(0.0)
        self._check(_lib.bbp_sweep(self._ctx, int(n), ctypes.byref(r)))
        return r.value

    def expect_site(self, x, y, op):
        op = np.ascontiguousarray(op, dtype=np.float64)
        out = ctypes.c_double()
        self._check(_lib.bbp_expect_site(self._ctx, x, y, _dptr(op),
                                         ctypes.byref(out)))
        return out.value

    def expect_bond(self, x0, y0, x1, y1, op):
        op = np.ascontiguousarray(op, dtype=np.float64)
        out = ctypes.c_double()
        self._check(_lib.bbp_expect_bond(self._ctx, x0, y0, x1, y1, _dptr(op),
                                         ctypes.byref(out)))
        return out.value

    def expect_sites(self, xs, ys, op):
        xs = np.ascontiguousarray(xs, dtype=np.int32)
        ys = np.ascontiguousarray(ys, dtype=np.int32)
        op = np.ascontiguousarray(op, dtype=np.float64)
        out = np.zeros(len(xs))
        self._check(_lib.bbp_expect_sites(self._ctx, len(xs), _iptr(xs),
                                          _iptr(ys), _dptr(op), _dptr(out)))
        return out

    def expect_bonds(self, bonds, op):
        b = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 4))
        cols = [np.ascontiguousarray(b[:, i]) for i in range(4)]
        op = np.ascontiguousarray(op, dtype=np.float64)
        out = np.zeros(len(b))
        self._check(_lib.bbp_expect_bonds(self._ctx, len(b),
                                          *[_iptr(c) for c in cols],
                                          _dptr(op), _dptr(out)))
        return out

    def expect_terms(self, xs, ys, op_site, bonds, op_bond):
        """Site values with op_site and bond values with op_bond from one
        call (bbp_expect_terms); returns (sites, bonds)."""
        xs = np.ascontiguousarray(xs, dtype=np.int32)
        ys = np.ascontiguousarray(ys, dtype=np.int32)
        b = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 4))
        cols = [np.ascontiguousarray(b[:, i]) for i in range(4)]
        op_site = np.ascontiguousarray(op_site, dtype=np.float64)
        op_bond = np.ascontiguousarray(op_bond, dtype=np.float64)
        out_s = np.zeros(len(xs))
        out_b = np.zeros(len(b))
        self._check(_lib.bbp_expect_terms(self._ctx, len(xs), _iptr(xs), _iptr(ys),
                                          _dptr(op_site), len(b),
                                          *[_iptr(c) for c in cols], _dptr(op_bond),
                                          _dptr(out_s), _dptr(out_b)))
        return out_s, out_b

    def rdm_sites(self, xs, ys):
        """One-site reduced density matrices, shape (n, d, d)."""
        xs = np.ascontiguousarray(xs, dtype=np.int32)
        ys = np.ascontiguousarray(ys, dtype=np.int32)
        d = self.d
        out = np.zeros((len(xs), d, d))
        self._check(_lib.bbp_rdm_sites(self._ctx, len(xs), _iptr(xs), _iptr(ys), _dptr(out)))
        return out

    def rdm_bonds(self, bonds):
        """Two-site reduced density matrices of bonds (x0, y0, x1, y1),
        shape (n, d^2, d^2)."""
        b = np.ascontiguousarray(np.asarray(bonds, dtype=np.int32).reshape(-1, 4))
        cols = [np.ascontiguousarray(b[:, k]) for k in range(4)]
        d2 = self.d * self.d
        out = np.zeros((len(b), d2, d2))
        self._check(_lib.bbp_rdm_bonds(self._ctx, len(b), *[_iptr(c) for c in cols],
                                       _dptr(out)))
        return out

    def ite_step(self, gate, n_als=4):
        """bbp_ite_step: one Trotter step of the blockBP update with the
        gate (d^2 x d^2) on every bond, the current messages fixed.  Returns
        (gates applied, summed relative fit error); ``self.ite_info`` holds
        the environment and host seconds and the number of gate levels."""
        g = np.ascontiguousarray(gate, dtype=np.float64).reshape(-1)
        if g.size != self.d ** 4:
            raise ValueError(f"gate needs {self.d ** 4} entries")
        info = np.zeros(5)
        self._check(_lib.bbp_ite_step(self._ctx, _dptr(g), int(n_als), _dptr(info)))
        self.ite_info = dict(env_s=float(info[2]), host_s=float(info[3]),
                             levels=int(info[4]))
        return int(info[0]), float(info[1])

    def log_norm(self):
        v = ctypes.c_double()
        s = ctypes.c_int32()
        self._check(_lib.bbp_log_norm(self._ctx, ctypes.byref(v),
                                      ctypes.byref(s)))
        return v.value, s.value

    def get_messages_flat(self):
        need = ctypes.c_size_t()
        self._check(_lib.bbp_get_messages(self._ctx, None, 0,
                                          ctypes.byref(need)))
        buf = np.zeros(need.value)
        self._check(_lib.bbp_get_messages(self._ctx, _dptr(buf), buf.size,
                                          ctypes.byref(need)))
        return buf

    def get_messages(self):
        """List of messages in enumeration order, each a list of site arrays
        ``[b_i, D*D, b_{i+1}]``."""
        buf = self.get_messages_flat()
        P = self.D * self.D
        out, o = [], 0
        while o < buf.size:
            n = int(buf[o])
            o += 1
            bonds = [int(v) for v in buf[o:o + n + 1]]
            o += n + 1
            m = []
            for s in range(n):
                size = bonds[s] * P * bonds[s + 1]
                m.append(buf[o:o + size].reshape(bonds[s], P, bonds[s + 1]))
                o += size
            out.append(m)
        return out

    def set_messages(self, msgs):
        parts = []
        for m in msgs:
            parts.append([float(len(m))])
            parts.append([1.0] + [float(t.shape[2]) for t in m])
            for t in m:
                parts.append(np.asarray(t, dtype=np.float64).reshape(-1))
        buf = np.ascontiguousarray(np.concatenate(parts))
        self._check(_lib.bbp_set_messages(self._ctx, _dptr(buf), buf.size))

    def stats(self):
        n = ctypes.c_int32()
        f = ctypes.c_double()
        self._check(_lib.bbp_stats(self._ctx, ctypes.byref(n), ctypes.byref(f)))
        return n.value, f.value

    def kernel_stats(self):
        """Per-kernel-class launch statistics (``timing`` option): list of
        dicts with name, launches, ms, flops and bytes (true extents,
        algorithmic), padded_flops and padded_bytes (bond cap, kernel data
        flow)."""
        out = []
        for i in range(9):
            name = ctypes.c_char_p()
            n = ctypes.c_int64()
            ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
            pf, pb = ctypes.c_double(), ctypes.c_double()
            self._check(_lib.bbp_kernel_stats(self._ctx, i, ctypes.byref(name),
                                              ctypes.byref(n), ctypes.byref(ms),
                                              ctypes.byref(fl), ctypes.byref(by)))
            self._check(_lib.bbp_kernel_stats_padded(self._ctx, i, ctypes.byref(pf),
                                                     ctypes.byref(pb)))
            out.append(dict(name=name.value.decode(), launches=n.value,
                            ms=ms.value, flops=fl.value, bytes=by.value,
                            padded_flops=pf.value, padded_bytes=pb.value))
        return out

    def kernel_stats_reset(self):
        self._check(_lib.bbp_kernel_stats_reset(self._ctx))

    def memory(self):
        """(bytes held now, most bytes held) on the device."""
        now, peak = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(_lib.bbp_memory(self._ctx, ctypes.byref(now), ctypes.byref(peak)))
        return now.value, peak.value

    def close(self):
        if self._ctx:
            _lib.bbp_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _request(Lx, Ly, bx, by, D, chi, tol=1e-10, max_sweeps=40,
             outputs=OUT_SZ | OUT_SS | OUT_LOGNORM, site_ops=(), bond_ops=()):
    return Request(Lx, Ly, bx, by, D, chi, max_sweeps, outputs, len(site_ops),
                   len(bond_ops), tol)


def estimate_bytes(**req):
    """bbp_server_estimate for a request given as keyword arguments."""
    n = ctypes.c_size_t()
    st = _lib.bbp_server_estimate(ctypes.byref(_request(**req)), ctypes.byref(n))
    if st != 0:
        raise BBPError(st, "malformed request")
    return n.value


def _update_args(H, W, D, chi, d, n_fit, seed, slot, A, mt, mr, mb):
    spec = UpdateSpec(H, W, D, d, chi, n_fit, seed, slot)
    S = chi * D * D * chi

    def side(m, n):
        if m is None:
            return None, None, None
        t, bonds = m
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() \
                or t.numel() < n * S:
            raise ValueError(f"a message needs {n} contiguous float64 device slots of {S}")
        b = np.ascontiguousarray(bonds, dtype=np.int32)
        if b.shape != (n + 1,):
            raise ValueError(f"a message of {n} sites needs {n + 1} bonds")
        return ctypes.c_void_p(t.data_ptr()), _iptr(b), b
    if A.dtype != torch.float64 or not A.is_cuda or not A.is_contiguous() \
            or A.numel() != H * W * d * D ** 4:
        raise ValueError(f"A must hold H*W*d*D^4 = {H * W * d * D ** 4} contiguous "
                         "float64 device values")
    out = torch.zeros(H * S, dtype=torch.float64, device=A.device)
    sides = [side(mt, W), side(mr, H), side(mb, W)]
    return spec, out, sides


NOALLOC_BYTES = 64 << 20   # BBP_UPDATE_NOALLOC_BYTES


def update_message(A, mt=None, mr=None, mb=None, *, H, W, D, chi, d=2, n_fit=2,
                   seed=0, slot=0, stream=None, noalloc=False):
    """bbp_update_message: one directed message update of an H x W block in
    the canonical frame (receiver on the left).  ``A``: device float64 tensor
    of the H*W rotated site tensors; ``mt``, ``mr``, ``mb``: ``(tensor,
    bonds)`` of the top, right and bottom messages in chi x D^2 x chi slots,
    or None (trivial).  Returns ``(out, bonds, log_scale)`` with ``out`` a
    device tensor of H slots.  ``noalloc``: bbp_update_message_noalloc (the
    library's static workspace; the output tensor is still allocated here, by
    the caller)."""
    spec, out, sides = _update_args(H, W, D, chi, d, n_fit, seed, slot, A, mt, mr, mb)
    bonds = np.zeros(H + 1, dtype=np.int32)
    ls = ctypes.c_double()
    handle = getattr(stream, "cuda_stream", stream)
    fn = _lib.bbp_update_message_noalloc if noalloc else _lib.bbp_update_message
    st = fn(ctypes.byref(spec), ctypes.c_void_p(A.data_ptr()),
                                 sides[0][0], sides[0][1], sides[1][0], sides[1][1],
                                 sides[2][0], sides[2][1], ctypes.c_void_p(out.data_ptr()),
                                 _iptr(bonds), ctypes.byref(ls), ctypes.c_void_p(handle))
    if st != 0:
        raise BBPError(st, _lib.bbp_update_last_error().decode())
    return out, bonds, ls.value


def trace_distance(rho, sigma):
    """bbp_trace_distance: Tr|rho - sigma| / 2 of two m x m real matrices."""
    a = np.ascontiguousarray(rho, dtype=np.float64)
    b = np.ascontiguousarray(sigma, dtype=np.float64)
    if a.ndim != 2 or a.shape[0] != a.shape[1] or a.shape != b.shape:
        raise ValueError("two square matrices of one size")
    out = ctypes.c_double()
    st = _lib.bbp_trace_distance(a.shape[0], _dptr(a), _dptr(b), ctypes.byref(out))
    if st != 0:
        raise BBPError(st, "bbp_trace_distance rejected its arguments")
    return out.value


SVD_MAX_WORDS = 19968   # BBP_SVD_MAX_WORDS


def svd_jacobi(A, k=None, *, max_sweeps=60, tol=0.0, stream=None):
    """bbp_svd_jacobi: truncated SVD of each m x n matrix of the float64
    device tensor ``A`` (batch, m, n), m >= n.  Returns device tensors
    ``(U (batch, m, k), S (batch, k), V (batch, n, k), err2 (batch,),
    sweeps (batch,))``; ``k`` defaults to n.  Enqueued on ``stream``
    (default: torch's current stream)."""
    if A.dtype != torch.float64 or not A.is_cuda or A.dim() != 3 or not A.is_contiguous():
        raise ValueError("A must be a contiguous float64 device tensor (batch, m, n)")
    b, m, n = A.shape
    k = n if k is None else int(k)
    dev = A.device
    U = torch.empty((b, m, k), dtype=torch.float64, device=dev)
    S = torch.empty((b, k), dtype=torch.float64, device=dev)
    V = torch.empty((b, n, k), dtype=torch.float64, device=dev)
    e2 = torch.empty((b,), dtype=torch.float64, device=dev)
    sw = torch.empty((b,), dtype=torch.int32, device=dev)
    if stream is None:
        stream = torch.cuda.current_stream(dev)
    handle = getattr(stream, "cuda_stream", stream)
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())
    st = _lib.bbp_svd_jacobi(b, m, n, k, ptr(A), ptr(U), ptr(S), ptr(V), ptr(e2), ptr(sw),
                             int(max_sweeps), float(tol), ctypes.c_void_p(handle))
    if st != 0:
        raise BBPError(st, "bbp_svd_jacobi rejected its arguments or the launch failed")
    return U, S, V, e2, sw


def ite_fit(N, theta, gate, D, n_als=4):
    """bbp_ite_fit: R[k, d, D], L[D, d, kb] fitted to gate . theta in the
    metric N[(k kb), (k kb)]; returns (R, L, relative fit error)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    k, d, _, kb = th.shape
    n = np.ascontiguousarray(N, dtype=np.float64).reshape(-1)
    g = np.ascontiguousarray(gate, dtype=np.float64).reshape(-1)
    if n.size != (k * kb) ** 2 or g.size != d ** 4:
        raise ValueError("N must be (k kb)^2 and the gate d^4 entries")
    R = np.zeros((k, d, D))
    L = np.zeros((D, d, kb))
    loss = ctypes.c_double()
    st = _lib.bbp_ite_fit(d, D, k, kb, _dptr(n), _dptr(th), _dptr(g), int(n_als),
                          _dptr(R), _dptr(L), ctypes.byref(loss))
    if st != 0:
        raise BBPError(st, "bbp_ite_fit rejected its arguments or the fit is singular")
    return R, L, loss.value


def update_workspace(H, W, D, chi, d=2, n_fit=2):
    """bbp_update_workspace: device bytes one update of this shape uses."""
    n = ctypes.c_size_t()
    st = _lib.bbp_update_workspace(ctypes.byref(UpdateSpec(H, W, D, d, chi, n_fit, 0, 0)),
                                   ctypes.byref(n))
    if st != 0:
        raise BBPError(st, _lib.bbp_update_last_error().decode())
    return n.value


def torch_allocator(device=None):
    """(alloc, free) over PyTorch's caching allocator, for
    ``BlockBP(allocator=...)``: the context's device memory then shows in
    torch.cuda.memory_allocated and is reused by torch after the context
    frees it."""
    import torch as _torch

    def alloc(nbytes):
        return _torch.cuda.caching_allocator_alloc(nbytes, device=device)

    def free(ptr):
        _torch.cuda.caching_allocator_delete(ptr)
    return alloc, free


class Server:
    """A libbbp request server (bbp_server_*).  ``submit`` takes the request
    as keyword arguments (Lx, Ly, bx, by, D, chi, tol, max_sweeps, outputs)
    and the site tensors; ``poll`` returns (state, result dict or None,
    (submit, admit, finish) times)."""

    def __init__(self, budget_bytes, max_slots):
        self._s = ctypes.c_void_p()
        st = _lib.bbp_server_create(ctypes.byref(self._s), int(budget_bytes),
                                    int(max_slots))
        if st != 0:
            raise BBPError(st, "bbp_server_create rejected its arguments")
        self._req = {}

    def submit(self, A, **req):
        """``site_ops`` / ``bond_ops``: sequences of 2x2 / 4x4 operators whose
        <O> on every site / bond the result lists (``site_op_values``,
        ``bond_op_values``)."""
        r = _request(**req)
        A = np.ascontiguousarray(A, dtype=np.float64)
        ops = [np.asarray(o, dtype=np.float64).reshape(-1) for o in req.get("site_ops", ())]
        ops += [np.asarray(o, dtype=np.float64).reshape(-1) for o in req.get("bond_ops", ())]
        flat = np.ascontiguousarray(np.concatenate(ops)) if ops else None
        t = ctypes.c_int64()
        st = _lib.bbp_server_submit(self._s, ctypes.byref(r), _dptr(A), A.size,
                                    _dptr(flat) if flat is not None else None,
                                    ctypes.byref(t))
        if st != 0:
            raise BBPError(st, "bbp_server_submit rejected the request")
        self._req[t.value] = r
        return t.value

    def poll(self, ticket):
        state = ctypes.c_int32()
        need = ctypes.c_size_t()
        times = np.zeros(3)
        st = _lib.bbp_server_poll(self._s, ticket, ctypes.byref(state), None, 0,
                                  ctypes.byref(need), _dptr(times))
        if st != 0:
            raise BBPError(st, "unknown ticket")
        if state.value != 2:
            return REQ_STATES[state.value], None, tuple(times)
        out = np.zeros(need.value)
        st = _lib.bbp_server_poll(self._s, ticket, ctypes.byref(state), _dptr(out),
                                  out.size, ctypes.byref(need), _dptr(times))
        if st != 0:
            raise BBPError(st, "poll")
        r = self._req[ticket]
        res = dict(converged=bool(out[0]), sweeps=int(out[1]), residual=out[2],
                   log_norm=out[3], sign=int(out[4]), peak_bytes=int(out[5]))
        o = 6
        if r.outputs & OUT_SZ:
            res["sz"] = out[o:o + r.Lx * r.Ly].reshape(r.Ly, r.Lx)
            o += r.Lx * r.Ly
        nb = (r.Lx - 1) * r.Ly + r.Lx * (r.Ly - 1)
        if r.outputs & OUT_SS:
            res["ss"] = out[o:o + nb]
            o += nb
        res["site_op_values"] = []
        for _ in range(r.n_site_ops):
            res["site_op_values"].append(out[o:o + r.Lx * r.Ly].reshape(r.Ly, r.Lx))
            o += r.Lx * r.Ly
        res["bond_op_values"] = []
        for _ in range(r.n_bond_ops):
            res["bond_op_values"].append(out[o:o + nb])
            o += nb
        return "done", res, tuple(times)

    def wait(self, ticket, timeout=600.0, interval=0.002):
        import time
        t0 = time.perf_counter()
        while True:
            state, res, times = self.poll(ticket)
            if state in ("done", "failed", "cancelled"):
                return state, res, times
            if time.perf_counter() - t0 > timeout:
                raise TimeoutError(f"request {ticket} still {state}")
            time.sleep(interval)

    def cancel(self, ticket):
        st = _lib.bbp_server_cancel(self._s, ticket)
        if st != 0:
            raise BBPError(st, "unknown ticket")

    def error(self, ticket):
        return _lib.bbp_server_error(self._s, ticket).decode()

    def stats(self):
        r, q, m = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        b = ctypes.c_size_t()
        st = _lib.bbp_server_stats(self._s, ctypes.byref(r), ctypes.byref(q),
                                   ctypes.byref(b), ctypes.byref(m))
        if st != 0:
            raise BBPError(st, "stats")
        sw, rs, mt = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        busy = np.zeros(3)
        st = _lib.bbp_server_sweeps(self._s, ctypes.byref(sw), ctypes.byref(rs),
                                    ctypes.byref(mt), _dptr(busy))
        if st != 0:
            raise BBPError(st, "sweeps")
        return dict(running=r.value, queued=q.value, bytes_in_use=b.value,
                    max_running=m.value, shared_sweeps=sw.value, request_sweeps=rs.value,
                    max_together=mt.value, sweep_s=busy[0], admit_s=busy[1],
                    outputs_s=busy[2])

    def close(self):
        if self._s:
            _lib.bbp_server_destroy(self._s)
            self._s = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
