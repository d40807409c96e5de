"""ctypes binding of libcrfrob.so (same names as include/crfrob.h).

Argument marshalling only: every step of the computation runs in the
library's host C++ and HIP kernels.  Loading fails loudly if the library is
missing; there is no fallback.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrfrob.so")

CR_OK, CR_EINVAL, CR_ENOTPRIME, CR_EPRANGE, CR_ESINGULAR, CR_ENOT_S_SMOOTH, \
    CR_EPRECISION, CR_ENOMEM, CR_EDEVICE, CR_ESELFCHECK = range(10)
CR_POLICY_DEPTH_FIRST, CR_POLICY_P_CHUNK, CR_POLICY_VAR_BY_VAR, CR_POLICY_LEARNED = range(4)

EXPORTS = ["cr_query_dims", "cr_monomials", "cr_precision", "cr_residue_words", "cr_check_smooth",
           "cr_frobenius_batch", "cr_frobenius", "cr_frobenius_batch_noalloc", "cr_newton_polygon", "cr_policy_cost",
           "cr_mlp_create", "cr_mlp_destroy", "cr_mlp_weights", "cr_mlp_forward", "cr_mlp_grad", "cr_mlp_train",
           "cr_trace_policy", "cr_autotune", "cr_autotune_cache", "cr_set_allocator", "cr_release", "cr_last_error"]

# hook types of cr_set_allocator: alloc(bytes, ctx) -> device pointer, free(ptr, ctx)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class cr_family(ctypes.Structure):
    _fields_ = [("nvars", ctypes.c_int32), ("degree", ctypes.c_int32), ("s_mask", ctypes.c_uint32),
                ("policy", ctypes.c_int32), ("r", ctypes.c_int32), ("n_series", ctypes.c_int32),
                ("engine", ctypes.c_int32), ("launch", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("M", ctypes.c_int32), ("n_series_m", ctypes.c_int32 * 6), ("grid", ctypes.c_int32)]


class cr_tuning(ctypes.Structure):
    _fields_ = [("best_policy", ctypes.c_int32), ("best_launch", ctypes.c_int32), ("best_ms", ctypes.c_double),
                ("ms", ctypes.c_double * 12), ("best_engine", ctypes.c_int32), ("best_grid", ctypes.c_int32),
                ("from_cache", ctypes.c_int32), ("shape_ms", ctypes.c_double * 8)]


class cr_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


CR_MLP_INPUTS, CR_MLP_HIDDEN, CR_MLP_PARAMS = 16, 128, 18817


CR_NEWTON_MAX = 256


class cr_newton(ctypes.Structure):
    _fields_ = [("b", ctypes.c_int32), ("nseg", ctypes.c_int32),
                ("seg_len", ctypes.c_int32 * CR_NEWTON_MAX), ("seg_rise", ctypes.c_int32 * CR_NEWTON_MAX),
                ("p_rank", ctypes.c_int32), ("ordinary", ctypes.c_int32), ("supersingular", ctypes.c_int32),
                ("height", ctypes.c_int32), ("domino_num", ctypes.c_int32), ("domino_den", ctypes.c_int32)]


class cr_stats(ctypes.Structure):
    _fields_ = [("start_blocks", ctypes.c_int64), ("column_steps", ctypes.c_int64),
                ("chunks", ctypes.c_int64), ("vectors", ctypes.c_int64),
                ("merged_terms", ctypes.c_int64), ("combined_groups", ctypes.c_int64),
                ("setup_ms", ctypes.c_double), ("device_ms", ctypes.c_double),
                ("reduce_ms", ctypes.c_double), ("combine_ms", ctypes.c_double),
                ("assemble_ms", ctypes.c_double), ("finish_ms", ctypes.c_double),
                ("engine", ctypes.c_int32), ("policy", ctypes.c_int32),
                ("phases", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("reduce_launches", ctypes.c_int64), ("psi_ms", ctypes.c_double)]


class CrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("crfrob status %d: %s" % (status, msg))
        self.status = status


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcrfrob.so is not built (run __graft_entry__.build()): %s" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        i32, u32, u64, i64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64
        L.cr_query_dims.argtypes = [i32, i32, P(i32), P(i32), P(i32)]
        L.cr_monomials.argtypes = [i32, i32, P(i32)]
        L.cr_precision.argtypes = [P(cr_family), i32, P(i32), P(i32), P(i32)]
        L.cr_residue_words.argtypes = [P(cr_family), i32, P(i32)]
        L.cr_check_smooth.argtypes = [P(cr_family), i32, P(u32), P(i32)]
        L.cr_frobenius.argtypes = [P(cr_family), i32, P(u32), P(u64), P(u64), P(i32), P(i32), P(i64),
                                   P(cr_stats), ctypes.c_void_p]
        L.cr_frobenius_batch.argtypes = [P(cr_family), i32, P(i32), P(u32), P(u64), P(u64), P(i32),
                                         P(i32), P(i64), P(i32), P(cr_stats), ctypes.c_void_p]
        L.cr_frobenius_batch_noalloc.argtypes = L.cr_frobenius_batch.argtypes
        L.cr_newton_polygon.argtypes = [i32, i32, i32, P(i64), P(cr_newton)]
        L.cr_policy_cost.argtypes = [P(cr_family), i32, P(u32), P(cr_stats)]
        f32, vp = ctypes.c_float, ctypes.c_void_p
        L.cr_mlp_create.argtypes = [P(f32), u64, P(vp)]
        L.cr_mlp_destroy.argtypes = [vp]
        L.cr_mlp_weights.argtypes = [vp, P(f32)]
        L.cr_mlp_forward.argtypes = [vp, i32, P(f32), P(f32), vp]
        L.cr_mlp_grad.argtypes = [vp, i32, P(f32), P(f32), P(f32), P(f32), vp]
        L.cr_mlp_train.argtypes = [vp, i32, P(f32), P(f32), P(cr_train_opts), P(f32), vp]
        L.cr_trace_policy.argtypes = [P(cr_family), i32, P(u32), i32, P(f32), P(f32), P(i32)]
        L.cr_autotune.argtypes = [P(cr_family), i32, P(i32), P(u32), i32, P(cr_tuning), vp]
        L.cr_autotune_cache.argtypes = [ctypes.c_char_p]
        L.cr_set_allocator.argtypes = [ALLOC_FN, FREE_FN, ctypes.c_void_p]
        L.cr_release.argtypes = []
        L.cr_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name != "cr_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st):
    if st != CR_OK:
        raise CrError(st, lib().cr_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


ENGINE_AUTO, ENGINE_VALU, ENGINE_MFMA_LDS, ENGINE_MFMA_SINGLE, ENGINE_QUAD, ENGINE_WIDE = 0, 1, 2, 3, 4, 5


LAUNCH_GRID, LAUNCH_PERSISTENT, LAUNCH_GRAPH = 0, 1, 2


def family(nvars, degree, s_mask=0, policy=CR_POLICY_DEPTH_FIRST, r=0, n_series=0, engine=ENGINE_AUTO, mlp=None,
           launch=LAUNCH_GRID, M=0, n_series_m=None, grid=0):
    """n_series_m: series orders N_m of pole orders m = 1..n (0 entries = n_series);
    grid: workgroups per CU of persistent launches (0 = 1)."""
    nm = list(n_series_m or []) + [0] * (6 - len(n_series_m or []))
    return cr_family(nvars, degree, s_mask, policy, r, n_series, engine, launch,
                     mlp.handle if mlp is not None else None, M, (ctypes.c_int32 * 6)(*nm), grid)


def cr_query_dims(nvars, degree):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().cr_query_dims(nvars, degree, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def cr_monomials(nvars, degree):
    nco = cr_query_dims(nvars, degree)[0]
    out = np.zeros((nco, nvars), dtype=np.int32)
    _check(lib().cr_monomials(nvars, degree, _ptr(out, ctypes.c_int32)))
    return out


def cr_precision(fam, p):
    r, N, M = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().cr_precision(ctypes.byref(fam), p, ctypes.byref(r), ctypes.byref(N), ctypes.byref(M)))
    return r.value, N.value, M.value


def cr_residue_words(fam, p):
    out = ctypes.c_int32()
    _check(lib().cr_residue_words(ctypes.byref(fam), p, ctypes.byref(out)))
    return out.value


def cr_check_smooth(fam, p, coeffs):
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint32))
    out = ctypes.c_int32()
    _check(lib().cr_check_smooth(ctypes.byref(fam), p, _ptr(c, ctypes.c_uint32), ctypes.byref(out)))
    return bool(out.value)


def _lpoly_ints(words):
    out = []
    for k in range(words.shape[0]):
        x = 0
        for j in range(4):
            x |= int(np.uint64(words[k, j])) << (64 * j)
        if x >> 255:
            x -= 1 << 256
        out.append(x)
    return out


def cr_frobenius_batch(fam, primes, coeffs, stream=None, want_scaled=True, raise_on_error=True, lpoly_ints=True,
                       noalloc=False):
    """Run the whole path for a batch; returns a dict of numpy arrays / lists.
    With lpoly_ints=False, "lpoly" is the raw (count, b+1, 4) array of 256-bit
    two's-complement words instead of lists of Python integers.  noalloc=True
    calls cr_frobenius_batch_noalloc (the static device workspace)."""
    primes = np.ascontiguousarray(np.asarray(primes, dtype=np.int32))
    count = int(primes.shape[0])
    nco, _s, b = cr_query_dims(fam.nvars, fam.degree)
    co = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint32).reshape(count, nco))
    frob = np.zeros((count, b, b), dtype=np.uint64)
    scaled = np.zeros((count, b, b), dtype=np.uint64) if want_scaled else None
    pole = np.zeros((count, b), dtype=np.int32)
    prec = np.zeros((count, b), dtype=np.int32)
    lp = np.zeros((count, b + 1, 4), dtype=np.int64)
    ist = np.zeros(count, dtype=np.int32)
    stats = cr_stats()
    fn = lib().cr_frobenius_batch_noalloc if noalloc else lib().cr_frobenius_batch
    st = fn(ctypes.byref(fam), count, _ptr(primes, ctypes.c_int32),
                                  _ptr(co, ctypes.c_uint32), _ptr(frob, ctypes.c_uint64),
                                  _ptr(scaled, ctypes.c_uint64) if scaled is not None else None,
                                  _ptr(pole, ctypes.c_int32), _ptr(prec, ctypes.c_int32),
                                  _ptr(lp, ctypes.c_int64), _ptr(ist, ctypes.c_int32),
                                  ctypes.byref(stats), ctypes.c_void_p(stream or 0))
    if raise_on_error:
        _check(st)
    return {
        "status": st, "item_status": ist, "frob": frob, "scaled": scaled, "col_pole": pole,
        "col_prec": prec, "lpoly": [_lpoly_ints(lp[i]) for i in range(count)] if lpoly_ints else lp, "stats": stats,
    }


def cr_frobenius(fam, p, coeffs, stream=None, want_scaled=True, raise_on_error=True):
    """One hypersurface; the same dict as cr_frobenius_batch, without the batch axis."""
    nco, _s, b = cr_query_dims(fam.nvars, fam.degree)
    co = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint32).reshape(nco))
    frob = np.zeros((b, b), dtype=np.uint64)
    scaled = np.zeros((b, b), dtype=np.uint64) if want_scaled else None
    pole = np.zeros(b, dtype=np.int32)
    prec = np.zeros(b, dtype=np.int32)
    lp = np.zeros((b + 1, 4), dtype=np.int64)
    stats = cr_stats()
    st = lib().cr_frobenius(ctypes.byref(fam), p, _ptr(co, ctypes.c_uint32), _ptr(frob, ctypes.c_uint64),
                            _ptr(scaled, ctypes.c_uint64) if scaled is not None else None,
                            _ptr(pole, ctypes.c_int32), _ptr(prec, ctypes.c_int32), _ptr(lp, ctypes.c_int64),
                            ctypes.byref(stats), ctypes.c_void_p(stream or 0))
    if raise_on_error:
        _check(st)
    return {"status": st, "frob": frob, "scaled": scaled, "col_pole": pole, "col_prec": prec,
            "lpoly": _lpoly_ints(lp), "stats": stats}


def lpoly_words(a):
    """Q(T) coefficients (Python integers) as the (b+1, 4) array of signed 256-bit
    two's-complement words that the library writes."""
    out = np.zeros((len(a), 4), dtype=np.int64)
    for i, x in enumerate(a):
        v = int(x) & ((1 << 256) - 1)
        for k in range(4):
            w = (v >> (64 * k)) & ((1 << 64) - 1)
            out[i, k] = w - (1 << 64) if w >= 1 << 63 else w
    return out


def cr_newton_polygon(nvars, degree, p, words, raise_on_error=True):
    """Newton-polygon invariants of Q(T) (host only): the cr_newton record, or
    None on error when raise_on_error is False."""
    w = np.ascontiguousarray(np.asarray(words, dtype=np.int64).reshape(-1, 4))
    out = cr_newton()
    st = lib().cr_newton_polygon(nvars, degree, p, _ptr(w, ctypes.c_int64), ctypes.byref(out))
    if st != CR_OK:
        if raise_on_error:
            _check(st)
        return None
    return out


def cr_policy_cost(fam, p, coeffs):
    """Host-only plan of one hypersurface under fam.policy: the cr_stats counters."""
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint32))
    stats = cr_stats()
    _check(lib().cr_policy_cost(ctypes.byref(fam), p, _ptr(c, ctypes.c_uint32), ctypes.byref(stats)))
    return stats


class Mlp:
    """Owner of a cr_mlp handle (the learned policy's network on the GPU)."""

    def __init__(self, weights=None, seed=0):
        h = ctypes.c_void_p()
        w = None
        if weights is not None:
            w = np.ascontiguousarray(np.asarray(weights, dtype=np.float32))
            assert w.shape == (CR_MLP_PARAMS,)
        _check(lib().cr_mlp_create(_ptr(w, ctypes.c_float) if w is not None else None, seed, ctypes.byref(h)))
        self.handle = h.value

    def close(self):
        if self.handle:
            lib().cr_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def weights(self):
        out = np.zeros(CR_MLP_PARAMS, dtype=np.float32)
        _check(lib().cr_mlp_weights(self.handle, _ptr(out, ctypes.c_float)))
        return out

    def forward(self, x, stream=None):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1, CR_MLP_INPUTS))
        y = np.zeros(x.shape[0], dtype=np.float32)
        _check(lib().cr_mlp_forward(self.handle, x.shape[0], _ptr(x, ctypes.c_float), _ptr(y, ctypes.c_float),
                                    ctypes.c_void_p(stream or 0)))
        return y

    def grad(self, x, t, stream=None):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1, CR_MLP_INPUTS))
        t = np.ascontiguousarray(np.asarray(t, dtype=np.float32))
        g = np.zeros(CR_MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().cr_mlp_grad(self.handle, x.shape[0], _ptr(x, ctypes.c_float), _ptr(t, ctypes.c_float),
                                 _ptr(g, ctypes.c_float), ctypes.byref(loss), ctypes.c_void_p(stream or 0)))
        return g, loss.value

    def train(self, x, t, epochs=10, batch=256, lr=0.0, seed=0, stream=None):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32).reshape(-1, CR_MLP_INPUTS))
        t = np.ascontiguousarray(np.asarray(t, dtype=np.float32))
        opts = cr_train_opts(epochs, batch, lr, 0.0, 0.0, 0.0, seed)
        losses = np.zeros(max(epochs, 1), dtype=np.float32)
        _check(lib().cr_mlp_train(self.handle, x.shape[0], _ptr(x, ctypes.c_float), _ptr(t, ctypes.c_float),
                                  ctypes.byref(opts), _ptr(losses, ctypes.c_float), ctypes.c_void_p(stream or 0)))
        return losses[:epochs]


def cr_trace_policy(fam, p, coeffs):
    """Training rows (inputs, labels) of one hypersurface's plain p-chunk plan."""
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint32))
    n = ctypes.c_int32()
    _check(lib().cr_trace_policy(ctypes.byref(fam), p, _ptr(c, ctypes.c_uint32), 0, None, None, ctypes.byref(n)))
    x = np.zeros((n.value, CR_MLP_INPUTS), dtype=np.float32)
    t = np.zeros(n.value, dtype=np.float32)
    _check(lib().cr_trace_policy(ctypes.byref(fam), p, _ptr(c, ctypes.c_uint32), n.value, _ptr(x, ctypes.c_float),
                                 _ptr(t, ctypes.c_float), ctypes.byref(n)))
    return x, t


def cr_autotune(fam, primes, coeffs, trials=2, stream=None):
    """Fastest (policy, launch) for this batch; returns the cr_tuning record."""
    primes = np.ascontiguousarray(np.asarray(primes, dtype=np.int32))
    nco = cr_query_dims(fam.nvars, fam.degree)[0]
    co = np.ascontiguousarray(np.asarray(coeffs, dtype=np.uint32).reshape(primes.shape[0], nco))
    out = cr_tuning()
    _check(lib().cr_autotune(ctypes.byref(fam), primes.shape[0], _ptr(primes, ctypes.c_int32),
                             _ptr(co, ctypes.c_uint32), trials, ctypes.byref(out), ctypes.c_void_p(stream or 0)))
    return out


def cr_autotune_cache(path):
    """Persist autotuner results in `path` (None: stop)."""
    _check(lib().cr_autotune_cache(path.encode() if path is not None else None))


_hook_errors = []  # exceptions raised inside the Python hooks (they cannot cross the C ABI)
_hooks = []  # every ctypes callback pair installed: blocks of live cr_mlp handles return through their own


def cr_set_allocator(alloc=None, free=None):
    """Install device-memory hooks: alloc(nbytes) -> device address (int, 0 on
    failure) and free(address); both None restores hipMalloc / hipFree."""
    if (alloc is None) != (free is None):
        raise ValueError("cr_set_allocator needs both hooks or neither")
    if alloc is None:
        _check(lib().cr_set_allocator(ALLOC_FN(), FREE_FN(), None))
        return
    def call_alloc(nbytes, _ctx):
        try:
            return int(alloc(int(nbytes))) or None
        except Exception as e:  # the library sees NULL (CR_ENOMEM)
            _hook_errors.append(e)
            return None

    def call_free(ptr, _ctx):
        try:
            free(int(ptr))
        except Exception as e:
            _hook_errors.append(e)

    a, f = ALLOC_FN(call_alloc), FREE_FN(call_free)
    _check(lib().cr_set_allocator(a, f, None))
    _hooks.append((a, f))


def cr_release():
    _check(lib().cr_release())
