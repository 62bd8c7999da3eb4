"""ctypes binding of libctm.so (argument marshalling only).

Every step of the split-CTMRG path runs inside the HIP library; this module
converts Python / NumPy / torch arguments into the plain pointers and sizes of
the C ABI in ``include/ctm.h`` and turns status codes into exceptions.  There
is no fallback: if the library is not built, loading raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_NAME = "libctm.so"

CTM_FP64, CTM_FP32, CTM_BF16 = 0, 1, 2
CTM_FLAG_DEVICE_PTRS = 1
CTM_FLAG_PROFILE = 2
CTM_FLAG_REDUCED = 4
CTM_FLAG_FULL_P4 = 8

STATUS = {0: "CTM_OK", 1: "CTM_EINVAL", 2: "CTM_ENOMEM", 3: "CTM_EDEVICE",
          4: "CTM_ENOCONV", 5: "CTM_ENUMERIC", 6: "CTM_ESTATE"}
CTM_OK, CTM_EINVAL, CTM_ENOMEM, CTM_EDEVICE, CTM_ENOCONV, CTM_ENUMERIC, CTM_ESTATE = range(7)


class CtmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int), ("chi", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("tol", ctypes.c_double), ("precision", ctypes.c_int), ("flags", ctypes.c_int),
                ("power_iters", ctypes.c_int), ("svd_cutoff", ctypes.c_double),
                ("lp_tol", ctypes.c_double), ("refine", ctypes.c_int)]


_LIB = None


def library_path():
    return os.environ.get("CTM_LIBRARY", os.path.join(_HERE, LIB_NAME))


def load_library(path=None):
    """Load libctm.so (raises OSError if it has not been built)."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or library_path()
    if not os.path.exists(p):
        raise OSError("HIP library %s not found: build it with __graft_entry__.build()" % p)
    # One HIP runtime per process: when PyTorch is installed its bundled
    # runtime (same soname) must be the one the library binds to, so torch is
    # imported first; loading the library first would pull in a second
    # runtime under torch.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(p)
    dp = ctypes.POINTER(ctypes.c_double)
    vp = ctypes.c_void_p
    lib.ctm_init.argtypes = [ctypes.POINTER(_Config), ctypes.c_double, vp, vp, ctypes.POINTER(vp)]
    lib.ctm_iterate.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp]
    lib.ctm_iterate_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), dp, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int)]
    lib.ctm_free_energy.argtypes = [vp, dp, dp, dp]
    lib.ctm_free_energy_noalloc.argtypes = [vp, dp, dp, dp]
    lib.ctm_grad.argtypes = [vp, vp]
    lib.ctm_magnetization.argtypes = [vp, dp]
    lib.ctm_bond_correlation.argtypes = [vp, dp]
    lib.ctm_energy.argtypes = [vp, dp]
    lib.ctm_corner_spectrum.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.ctm_reset_tensor.argtypes = [vp, ctypes.c_double, vp]
    lib.ctm_query.argtypes = [vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_longlong)]
    lib.ctm_kernel_stats.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong), dp, dp, dp]
    lib.ctm_kernel_stats.restype = ctypes.c_int
    lib.ctm_destroy.argtypes = [vp]
    lib.ctm_destroy.restype = None
    lib.ctm_last_error.argtypes = [vp]
    lib.ctm_last_error.restype = ctypes.c_char_p
    lib.ctm_status_string.argtypes = [ctypes.c_int]
    lib.ctm_status_string.restype = ctypes.c_char_p
    lib.ctm_abi_version.restype = ctypes.c_int
    for fn in ("ctm_init", "ctm_iterate", "ctm_iterate_batch", "ctm_free_energy", "ctm_free_energy_noalloc",
               "ctm_grad", "ctm_corner_spectrum",
               "ctm_reset_tensor", "ctm_query"):
        getattr(lib, fn).restype = ctypes.c_int
    if path is None:
        _LIB = lib
    return lib


def abi_version(lib=None):
    return (lib or load_library()).ctm_abi_version()


def _host_f64(A):
    a = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
    return a, a.ctypes.data_as(ctypes.c_void_p)


class SplitCTM:
    """One context: both networks (triple and double layer) for one (beta, A).

    ``A`` is a float64 array of shape (2, D, D, D, D) ([p][l][u][r][d]); a torch
    tensor on the GPU is passed by device pointer.  ``stream`` is a HIP stream
    handle (int) or None for the default stream.  ``method="reduced"`` contracts
    both networks with the reduced (fused-site, C4v) CTMRG instead of
    split-CTMRG (CTM_FLAG_REDUCED; FP64 only).
    """

    def __init__(self, beta, A, chi, max_iter=100, tol=0.0, precision=CTM_FP64,
                 power_iters=0, svd_cutoff=0.0, stream=None, lib=None, profile=False,
                 lp_tol=0.0, refine=False, method="split", p4="half"):
        if method not in ("split", "reduced"):
            raise ValueError("method must be 'split' or 'reduced'")
        self._lib = lib or load_library()
        self._ctx = ctypes.c_void_p()
        D = int(np.shape(A)[1])
        flags, ptr, keep = self._tensor_arg(A)
        if profile:
            flags |= CTM_FLAG_PROFILE
        if method == "reduced":
            flags |= CTM_FLAG_REDUCED
        if p4 not in ("full", "half"):
            raise ValueError("p4 must be 'full' or 'half'")
        if p4 == "full":
            flags |= CTM_FLAG_FULL_P4
        cfg = _Config(D, int(chi), int(max_iter), float(tol), int(precision), flags,
                      int(power_iters), float(svd_cutoff), float(lp_tol), int(bool(refine)))
        st = self._lib.ctm_init(ctypes.byref(cfg), float(beta), ptr,
                                ctypes.c_void_p(stream or 0), ctypes.byref(self._ctx))
        del keep
        if st != 0:
            raise CtmError(st, self._lib.ctm_last_error(None).decode())
        self.D, self.chi, self.beta, self._flags = D, int(chi), float(beta), flags

    @staticmethod
    def _tensor_arg(A):
        if hasattr(A, "is_cuda") and A.is_cuda:
            import torch
            if A.dtype != torch.float64 or not A.is_contiguous():
                raise TypeError("device A must be a contiguous float64 tensor")
            return CTM_FLAG_DEVICE_PTRS, ctypes.c_void_p(A.data_ptr()), A
        a, p = _host_f64(A)
        return 0, p, a

    def _check(self, st, allow=()):
        if st != 0 and st not in allow:
            raise CtmError(st, self._lib.ctm_last_error(self._ctx).decode())
        return st

    def iterate(self, n_iter=0, allow_noconv=True):
        done = ctypes.c_int(0)
        dl = ctypes.c_double(0.0)
        st = self._lib.ctm_iterate(self._ctx, int(n_iter), ctypes.byref(done), ctypes.byref(dl))
        self._check(st, allow=(CTM_ENOCONV,) if allow_noconv else ())
        return done.value, dl.value, st == 0

    def free_energy(self):
        f, k3, k2 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.ctm_free_energy(self._ctx, ctypes.byref(f), ctypes.byref(k3), ctypes.byref(k2)))
        return f.value, k3.value, k2.value

    def free_energy_noalloc(self):
        """free_energy() with the library's fixed scratch (ctm_free_energy_noalloc)."""
        f, k3, k2 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._lib.ctm_free_energy_noalloc(self._ctx, ctypes.byref(f), ctypes.byref(k3),
                                                      ctypes.byref(k2)))
        return f.value, k3.value, k2.value

    def grad(self, out=None):
        n = 2 * self.D ** 4
        if out is not None and hasattr(out, "is_cuda") and out.is_cuda:
            if not (self._flags & CTM_FLAG_DEVICE_PTRS):
                raise ValueError("device output needs a context built from a device tensor")
            self._check(self._lib.ctm_grad(self._ctx, ctypes.c_void_p(out.data_ptr())))
            return out
        g = np.empty((2,) + (self.D,) * 4)
        if self._flags & CTM_FLAG_DEVICE_PTRS:
            raise ValueError("a device context needs a device output tensor")
        self._check(self._lib.ctm_grad(self._ctx, g.ctypes.data_as(ctypes.c_void_p)))
        assert g.size == n
        return g

    def magnetization(self):
        """<sigma> of a PEPO-layer spin in the converged triple-layer environment."""
        m = ctypes.c_double()
        self._check(self._lib.ctm_magnetization(self._ctx, ctypes.byref(m)))
        return m.value

    def bond_correlation(self):
        """In-plane nearest-neighbour <sigma sigma'> of two PEPO-layer spins."""
        zz = ctypes.c_double()
        self._check(self._lib.ctm_bond_correlation(self._ctx, ctypes.byref(zz)))
        return zz.value

    def energy(self):
        """Internal energy per site U = -d ln kappa3 / d beta at fixed A."""
        u = ctypes.c_double()
        self._check(self._lib.ctm_energy(self._ctx, ctypes.byref(u)))
        return u.value

    def spectrum(self, which=3):
        cap = 4096
        buf = (ctypes.c_double * cap)()
        n = ctypes.c_int(0)
        self._check(self._lib.ctm_corner_spectrum(self._ctx, int(which), buf, cap, ctypes.byref(n)))
        return np.array(buf[: n.value])

    def reset_tensor(self, beta, A):
        flags, ptr, keep = self._tensor_arg(A)
        if flags != (self._flags & CTM_FLAG_DEVICE_PTRS):
            raise ValueError("A must live where the context's A lived (host vs device)")
        self._check(self._lib.ctm_reset_tensor(self._ctx, float(beta), ptr))
        self.beta = float(beta)

    def kernel_stats(self, which):
        """(launches, total ms, algorithmic flops, algorithmic bytes) of kernel
        class which (0 FP64 GEMM, 1 Jacobi, 2 Cholesky QR, 3 FP32/BF16 GEMM,
        4 split-K reduction, 5 the factorisations' part of class 0) of a
        context built with profile=True."""
        n = ctypes.c_longlong(0)
        ms = ctypes.c_double(0.0)
        fl = ctypes.c_double(0.0)
        by = ctypes.c_double(0.0)
        self._check(self._lib.ctm_kernel_stats(self._ctx, int(which), ctypes.byref(n), ctypes.byref(ms),
                                               ctypes.byref(fl), ctypes.byref(by)))
        return n.value, ms.value, fl.value, by.value

    def query(self):
        it = ctypes.c_int(0)
        b = ctypes.c_longlong(0)
        self._check(self._lib.ctm_query(self._ctx, ctypes.byref(it), ctypes.byref(b)))
        return it.value, b.value

    def close(self):
        if self._ctx:
            self._lib.ctm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def iterate_batch(contexts, n_iter=0, lib=None):
    """Advance several SplitCTM contexts together (ctm_iterate_batch): one move
    of every still-active context per step, the networks of all of them
    running concurrently.  n_iter as in ``SplitCTM.iterate`` (negative: a
    slice of at most -n_iter moves with the stopping rule).  Returns
    [(iters_done, last_delta, converged, status)] per context; raises only for
    argument errors (CTM_EINVAL)."""
    n = len(contexts)
    if n == 0:
        return []
    lib = lib or contexts[0]._lib
    arr = (ctypes.c_void_p * n)(*[c._ctx.value for c in contexts])
    done = (ctypes.c_int * n)()
    dl = (ctypes.c_double * n)()
    cv = (ctypes.c_int * n)()
    st = (ctypes.c_int * n)()
    s = lib.ctm_iterate_batch(arr, n, int(n_iter), done, dl, cv, st)
    if s == 1:
        raise CtmError(s, "ctm_iterate_batch: invalid arguments")
    return [(done[i], dl[i], bool(cv[i]), st[i]) for i in range(n)]
