"""Python binding of libfepll.so, the gfx950 EPLL denoising library.

Argument marshalling only: every step of the restoration runs in the HIP
kernels behind the C ABI declared in include/fepll.h.  PyTorch supplies
device memory and the current stream.  There is no fallback: if the shared
library is missing, importing the binding's functions raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

__all__ = ["FepllError", "GMM", "cov_eig", "restore", "restore_batch", "autotune", "set_tuning",
           "get_tuning", "select", "profile", "library_path", "FP32", "BF16", "FP8"]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfepll.so")

FP32, BF16, FP8 = 0, 1, 2
_PREC = {"fp32": FP32, "bf16": BF16, "fp8": FP8}
_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EUNSUPPORTED",
           -5: "ECHECKSUM"}


class FepllError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class Image(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("height", c_int32), ("width", c_int32),
                ("row_stride", c_int64), ("on_device", c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("recheck", c_int32), ("use_proposal", c_int32),
                ("top_m", c_int32), ("margin_nats", c_double), ("init", POINTER(Image)),
                ("stream", c_void_p), ("profile", c_int32), ("jitter", c_int32),
                ("seed", ctypes.c_uint64), ("use_tree", c_int32)]


class Operator(ctypes.Structure):
    """fepll_operator: the degradation A (kind 0 identity, 1 periodic
    convolution with a centred odd-sized float32 kernel)."""
    _fields_ = [("kind", c_int32), ("kh", c_int32), ("kw", c_int32), ("kernel", c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("est_blocks", c_int32), ("wiener_blocks", c_int32), ("ola_rows", c_int32),
                ("reserved", c_int32)]


class AdamW(ctypes.Structure):
    _fields_ = [("lr", c_double), ("beta1", c_double), ("beta2", c_double), ("eps", c_double),
                ("weight_decay", c_double)]


_lib = None


def library_path() -> str:
    return LIB_PATH


def lib():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    L.fepll_options_default.argtypes = [POINTER(Options)]
    L.fepll_options_default.restype = None
    L.fepll_last_error.restype = c_char_p
    L.fepll_version.restype = c_char_p
    L.fepll_gmm_create.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                   POINTER(c_void_p)]
    L.fepll_gmm_create.restype = c_int32
    L.fepll_gmm_create_from_cov.argtypes = [c_void_p, c_void_p, c_int32, c_int32,
                                            POINTER(c_void_p)]
    L.fepll_gmm_create_from_cov.restype = c_int32
    L.fepll_cov_eig.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p]
    L.fepll_cov_eig.restype = c_int32
    L.fepll_gmm_destroy.argtypes = [c_void_p]
    L.fepll_gmm_destroy.restype = None
    L.fepll_gmm_flat_tail.argtypes = [c_void_p, c_double, c_void_p]
    L.fepll_gmm_flat_tail.restype = c_int32
    L.fepll_gmm_set_tree.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
    L.fepll_gmm_set_tree.restype = c_int32
    L.fepll_restore.argtypes = [c_void_p, POINTER(Image), c_void_p, c_double, c_void_p, c_int32,
                                POINTER(Image), POINTER(Options), c_void_p]
    L.fepll_restore.restype = c_int32
    L.fepll_restore_batch.argtypes = [c_void_p, c_int32, POINTER(Image), c_void_p,
                                      POINTER(Image), POINTER(Options)]
    L.fepll_restore_batch.restype = c_int32
    L.fepll_set_tuning.argtypes = [c_void_p, POINTER(Tuning)]
    L.fepll_set_tuning.restype = c_int32
    L.fepll_get_tuning.argtypes = [c_void_p, POINTER(Tuning)]
    L.fepll_get_tuning.restype = c_int32
    L.fepll_autotune.argtypes = [c_void_p, c_int32, POINTER(Image), c_void_p, POINTER(Options),
                                 POINTER(Tuning)]
    L.fepll_autotune.restype = c_int32
    L.fepll_select.argtypes = [c_void_p, POINTER(Image), c_double, c_void_p, c_void_p, c_void_p,
                               c_void_p, POINTER(Options)]
    L.fepll_select.restype = c_int32
    L.fepll_select_static.argtypes = [c_void_p, POINTER(Image), c_double, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p]
    L.fepll_select_static.restype = c_int32
    L.fepll_set_memory_limit.argtypes = [ctypes.c_size_t]
    L.fepll_set_memory_limit.restype = c_int32
    L.fepll_memory_in_use.argtypes = []
    L.fepll_memory_in_use.restype = ctypes.c_size_t
    L.fepll_profile.argtypes = [c_void_p, POINTER(c_double), POINTER(c_int32), c_int32]
    L.fepll_profile.restype = c_int32
    L.fepll_mlp_param_count.argtypes = [c_int32]
    L.fepll_mlp_param_count.restype = c_int64
    L.fepll_mlp_create.argtypes = [c_int32, c_void_p, c_int32, POINTER(c_void_p)]
    L.fepll_mlp_create.restype = c_int32
    L.fepll_mlp_destroy.argtypes = [c_void_p]
    L.fepll_mlp_destroy.restype = None
    L.fepll_mlp_get_params.argtypes = [c_void_p, c_void_p]
    L.fepll_mlp_get_params.restype = c_int32
    L.fepll_mlp_forward.argtypes = [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]
    L.fepll_mlp_forward.restype = c_int32
    L.fepll_mlp_loss_grad.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_void_p,
                                      c_void_p]
    L.fepll_mlp_loss_grad.restype = c_int32
    L.fepll_mlp_train_step.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int32,
                                       POINTER(AdamW), c_void_p, c_void_p]
    L.fepll_mlp_train_step.restype = c_int32
    L.fepll_features.argtypes = [POINTER(Image), c_double, c_void_p, c_void_p]
    L.fepll_features.restype = c_int32
    L.fepll_mlp_serialize.argtypes = [c_void_p, c_void_p, ctypes.c_size_t,
                                      POINTER(ctypes.c_size_t)]
    L.fepll_mlp_serialize.restype = c_int32
    L.fepll_gmm_load_proposal.argtypes = [c_void_p, c_void_p, ctypes.c_size_t]
    L.fepll_gmm_load_proposal.restype = c_int32
    L.fepll_propose.argtypes = [c_void_p, POINTER(Image), c_double, c_int32, c_void_p, c_void_p]
    L.fepll_propose.restype = c_int32
    _lib = L
    return L


def _check(st: int):
    if st != 0:
        raise FepllError(st, lib().fepll_last_error().decode())


def _ptr(a) -> int:
    """Data pointer of a torch tensor or a C-contiguous numpy array."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _image(t) -> Image:
    import torch
    if isinstance(t, np.ndarray):
        if t.dtype != np.float32 or t.ndim != 2 or t.strides[1] != 4:
            raise ValueError("image must be a 2-D float32 array with unit column stride")
        return Image(t.ctypes.data, t.shape[0], t.shape[1], t.strides[0] // 4, 0)
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.dim() != 2 \
            or t.stride(1) != 1:
        raise ValueError("image must be a 2-D float32 tensor with unit column stride")
    return Image(t.data_ptr(), t.shape[0], t.shape[1], t.stride(0), 1 if t.is_cuda else 0)


STAGES = ("select", "recheck", "bucket", "wiener", "ola_update", "prep", "propose", "fallback",
          "subset")


def _options(precision="fp32", recheck=True, init=None, stream=None, profile=False,
             proposal=False, top_m=8, margin=0.5, jitter=0, seed=0, tree=False) -> Options:
    o = Options()
    lib().fepll_options_default(ctypes.byref(o))
    o.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    o.recheck = 1 if recheck else 0
    if init is not None:
        o._init_img = _image(init)  # keep alive with the struct
        o.init = ctypes.pointer(o._init_img)
    o.stream = stream
    # stage timing: False, True (every stage), a list of stage names, or the
    # raw options.profile value (an int)
    if isinstance(profile, (list, tuple)):
        o.profile = sum(2 << STAGES.index(st) for st in profile)
    elif isinstance(profile, int) and not isinstance(profile, bool):
        o.profile = profile
    else:
        o.profile = 1 if profile else 0
    o.use_proposal = 1 if proposal else 0
    o.top_m = int(top_m)
    o.margin_nats = float(margin)
    o.jitter = int(jitter)
    o.seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    o.use_tree = 1 if tree else 0
    return o


def _stream_of(t):
    import torch
    if isinstance(t, torch.Tensor) and t.is_cuda:
        return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)
    return None


class GMM:
    """Device-resident mixture: U (K,64,64) eigenvectors as columns,
    lam (K,64) eigenvalues, w (K,) weights -- all float64 on the host."""

    def __init__(self, U, lam, w):
        U = np.ascontiguousarray(U, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        K = w.shape[0]
        if U.shape != (K, 64, 64) or lam.shape != (K, 64):
            raise ValueError("U must be (K,64,64), lam (K,64), w (K,)")
        h = c_void_p()
        _check(lib().fepll_gmm_create(U.ctypes.data, lam.ctypes.data, w.ctypes.data, K, 64,
                                      ctypes.byref(h)))
        self._h = h
        self.K = K

    @classmethod
    def from_cov(cls, Sigma, w):
        """Mixture from its covariances Sigma (K,64,64) and weights w (K,),
        float64; the eigendecomposition runs in the library."""
        Sigma = np.ascontiguousarray(Sigma, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        K = w.shape[0]
        if Sigma.shape != (K, 64, 64):
            raise ValueError("Sigma must be (K,64,64), w (K,)")
        self = cls.__new__(cls)
        h = c_void_p()
        _check(lib().fepll_gmm_create_from_cov(Sigma.ctypes.data, w.ctypes.data, K, 64,
                                               ctypes.byref(h)))
        self._h = h
        self.K = K
        return self

    @property
    def handle(self):
        return self._h

    def flat_tail(self, rho: float) -> np.ndarray:
        """Flat-tail spectrum approximation (Sec. 3.1) for later calls:
        returns the kept ranks r_k (K,) int32; rho = 1 turns it off."""
        r = np.empty(self.K, dtype=np.int32)
        _check(lib().fepll_gmm_flat_tail(self._h, float(rho), r.ctypes.data))
        return r

    def set_tree(self, sizes, parents):
        """Search tree for the selection (Sec. 3.2): level sizes, root first
        (1, ..., K), and per level below the root the parent of each node in
        the level above (e.g. from paper_1710_08124_amd.tree.build_tree).
        sizes = None removes the tree."""
        if sizes is None:
            _check(lib().fepll_gmm_set_tree(self._h, 0, None, None))
            return
        sz = np.ascontiguousarray(sizes, dtype=np.int32)
        if len(parents) != sz.size - 1:
            raise ValueError("one parent array per level below the root")
        for n, p in enumerate(parents):
            if np.asarray(p).shape != (int(sz[n + 1]),):
                raise ValueError("parents[n] must hold one entry per node of level n + 1")
        par = np.ascontiguousarray(np.concatenate([np.asarray(p, np.int32) for p in parents]))
        _check(lib().fepll_gmm_set_tree(self._h, int(sz.size), sz.ctypes.data, par.ctypes.data))

    def load_proposal(self, blob: bytes):
        """Attach a serialized proposal network (see MLP.serialize)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(lib().fepll_gmm_load_proposal(self._h, buf, len(blob)))

    def close(self):
        if getattr(self, "_h", None):
            lib().fepll_gmm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cov_eig(Sigma):
    """(U, lam) with Sigma[k] = U[k] diag(lam[k]) U[k]^t, lam decreasing:
    the library's float64 eigendecomposition (host only)."""
    Sigma = np.ascontiguousarray(Sigma, dtype=np.float64)
    K, d, _ = Sigma.shape
    U = np.empty((K, d, d))
    lam = np.empty((K, d))
    _check(lib().fepll_cov_eig(Sigma.ctypes.data, K, d, U.ctypes.data, lam.ctypes.data))
    return U, lam


def profile(gmm: GMM):
    """Stage times (ms) and launch counts accumulated since the last read."""
    ns = len(STAGES)
    ms = (c_double * ns)()
    n = (c_int32 * ns)()
    _check(lib().fepll_profile(gmm.handle, ms, n, ns))
    return {s: (ms[i], n[i]) for i, s in enumerate(STAGES)}


def restore(gmm: GMM, y, sigma: float, betas=None, init=None, precision="fp32",
            recheck=True, return_labels=False, out=None, profile=False, proposal=False,
            top_m=8, margin=0.5, jitter=0, seed=0, blur=None, tree=False):
    """Denoise y (2-D float32 torch tensor, CUDA or CPU, or numpy array).

    betas: absolute beta values (default {1,4,8,16,32}/sigma^2).
    jitter: 0, or the grid spacing s of the jittered patch subsampling
    (Sec. 3.3) with its Philox seed.
    tree: select through the search tree of gmm.set_tree (Sec. 3.2; bf16).
    blur: None (denoising), or the centred odd-sized kernel of a periodic
    convolution A (deblurring; the Sec. 5 schedule and start by default).
    Returns the restored image (same kind and device as y) and, with
    return_labels, the (T, Np) int32 labels of every iteration (K for the
    patches an iteration did not choose).
    """
    import torch
    yi = _image(y)
    if out is None:
        out = torch.empty_like(y) if isinstance(y, torch.Tensor) else np.empty_like(y)
    oi = _image(out)
    o = _options(precision, recheck, init, _stream_of(y), profile, proposal, top_m, margin,
                 jitter, seed, tree)
    if betas is None:
        bptr, T = None, 0
        Tn = 5
    else:
        b = np.ascontiguousarray(betas, dtype=np.float64)
        bptr, T = b.ctypes.data, b.size
        Tn = T
    labels = None
    lptr = None
    if return_labels:
        Np = (y.shape[0] - 7) * (y.shape[1] - 7)
        if isinstance(y, torch.Tensor):
            labels = torch.empty((Tn, Np), dtype=torch.int32, device=y.device)
        else:
            labels = np.empty((Tn, Np), dtype=np.int32)
        lptr = _ptr(labels)
    op = None
    if blur is not None:
        k = np.ascontiguousarray(blur, dtype=np.float32)
        if k.ndim != 2:
            raise ValueError("blur must be a 2-D kernel")
        op = Operator(1, k.shape[0], k.shape[1], k.ctypes.data)
        op._keep = k
    _check(lib().fepll_restore(gmm.handle, ctypes.byref(yi),
                               ctypes.byref(op) if op is not None else None, float(sigma), bptr, T,
                               ctypes.byref(oi), ctypes.byref(o), lptr))
    return (out, labels) if return_labels else out


def _batch_args(ys, sigmas, outs):
    import torch
    n = len(ys)
    if len(sigmas) != n:
        raise ValueError("one sigma per image")
    if outs is None:
        outs = [torch.empty_like(y) if isinstance(y, torch.Tensor) else np.empty_like(y)
                for y in ys]
    yi = (Image * n)(*[_image(y) for y in ys])
    oi = (Image * n)(*[_image(o) for o in outs])
    sg = np.ascontiguousarray(sigmas, dtype=np.float64)
    return n, yi, oi, sg, outs


def restore_batch(gmm: GMM, ys, sigmas, precision="bf16", recheck=True, outs=None,
                  profile=False, proposal=False, top_m=8, margin=0.5, jitter=0, seed=0,
                  tree=False):
    """Denoise a list of images (2-D float32 tensors or arrays, any sizes),
    each with its own noise level, in one batched call (default schedule).
    Returns the list of restored images."""
    n, yi, oi, sg, outs = _batch_args(ys, sigmas, outs)
    o = _options(precision, recheck, None, _stream_of(ys[0]), profile, proposal, top_m, margin,
                 jitter, seed, tree)
    _check(lib().fepll_restore_batch(gmm.handle, n, yi, sg.ctypes.data, oi, ctypes.byref(o)))
    return outs


def set_tuning(gmm: GMM, est_blocks=768, wiener_blocks=4096, ola_rows=16):
    t = Tuning(int(est_blocks), int(wiener_blocks), int(ola_rows), 0)
    _check(lib().fepll_set_tuning(gmm.handle, ctypes.byref(t)))


def get_tuning(gmm: GMM) -> dict:
    t = Tuning()
    _check(lib().fepll_get_tuning(gmm.handle, ctypes.byref(t)))
    return {"est_blocks": t.est_blocks, "wiener_blocks": t.wiener_blocks,
            "ola_rows": t.ola_rows}


def autotune(gmm: GMM, ys, sigmas, precision="bf16", proposal=False, top_m=8, margin=0.5):
    """Time the candidate launch shapes on this batch, keep the fastest in
    the handle and return them."""
    n, yi, _, sg, _ = _batch_args(ys, sigmas, [ys[0]] * len(ys))
    o = _options(precision, True, None, _stream_of(ys[0]), False, proposal, top_m, margin)
    t = Tuning()
    _check(lib().fepll_autotune(gmm.handle, n, yi, sg.ctypes.data, ctypes.byref(o),
                                ctypes.byref(t)))
    return get_tuning(gmm)


def select(gmm: GMM, x, beta: float, recheck=True, precision="fp32", proposal=False, top_m=8,
           margin=0.5, tree=False):
    """One Gaussian-selection step on the CUDA image x.
    Returns (labels int32, best f32, second f32, flags int32), each of
    length (H-7)*(W-7)."""
    import torch
    xi = _image(x)
    Np = (x.shape[0] - 7) * (x.shape[1] - 7)
    dev = x.device
    lab = torch.empty(Np, dtype=torch.int32, device=dev)
    best = torch.empty(Np, dtype=torch.float32, device=dev)
    second = torch.empty(Np, dtype=torch.float32, device=dev)
    flags = torch.empty(Np, dtype=torch.int32, device=dev)
    o = _options(precision, recheck, None, _stream_of(x), False, proposal, top_m, margin,
                 tree=tree)
    _check(lib().fepll_select(gmm.handle, ctypes.byref(xi), float(beta), lab.data_ptr(),
                              best.data_ptr(), second.data_ptr(), flags.data_ptr(),
                              ctypes.byref(o)))
    return lab, best, second, flags


def set_memory_limit(limit_bytes: int):
    """Cap on the device memory the library holds (0: none); allocations
    past it fail with ENOMEM."""
    _check(lib().fepll_set_memory_limit(int(limit_bytes)))


def memory_in_use() -> int:
    """Bytes of device memory the library holds."""
    return int(lib().fepll_memory_in_use())


def select_static(gmm: GMM, x, beta: float, out=None):
    """fepll_select_static: the float32 selection of select() without device
    allocation inside the library, on the contiguous CUDA image x.  out: a
    tuple (labels, best, second, flags) of preallocated CUDA tensors of
    (H-7)*(W-7) entries (int32, float32, float32, int32), or None (allocated
    here by PyTorch).  Returns the four tensors."""
    import torch
    xi = _image(x)
    Np = (x.shape[0] - 7) * (x.shape[1] - 7)
    if out is None:
        dev = x.device
        out = (torch.empty(Np, dtype=torch.int32, device=dev),
               torch.empty(Np, dtype=torch.float32, device=dev),
               torch.empty(Np, dtype=torch.float32, device=dev),
               torch.empty(Np, dtype=torch.int32, device=dev))
    lab, best, second, flags = out
    _check(lib().fepll_select_static(gmm.handle, ctypes.byref(xi), float(beta), lab.data_ptr(),
                                     best.data_ptr(), second.data_ptr(), flags.data_ptr(),
                                     _stream_of(x)))
    return lab, best, second, flags


def propose(gmm: GMM, x, beta: float, top_m: int = 8):
    """Candidates of the attached network for every patch of the CUDA image x:
    (Np, 8) int32, -1 after the top_m-th."""
    import torch
    xi = _image(x)
    Np = (x.shape[0] - 7) * (x.shape[1] - 7)
    cand = torch.empty((Np, 8), dtype=torch.int16, device=x.device)
    _check(lib().fepll_propose(gmm.handle, ctypes.byref(xi), float(beta), int(top_m),
                               cand.data_ptr(), _stream_of(x)))
    c = cand.to(torch.int32) & 0xFFFF
    c[c == 0xFFFF] = -1
    return c


def features(x, beta: float):
    """Network input [z~/128, log sigma_beta] of every patch of CUDA image x."""
    import torch
    xi = _image(x)
    Np = (x.shape[0] - 7) * (x.shape[1] - 7)
    X = torch.empty((Np, 65), dtype=torch.float32, device=x.device)
    _check(lib().fepll_features(ctypes.byref(xi), float(beta), X.data_ptr(), _stream_of(x)))
    return X


PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten_params(p: dict) -> np.ndarray:
    """W1 b1 W2 b2 W3 b3 (W as (out, in)) into one float32 vector."""
    return np.concatenate([np.asarray(p[k], np.float32).ravel() for k in PARAM_NAMES])


def unflatten_params(v: np.ndarray, K: int) -> dict:
    shapes = {"W1": (256, 65), "b1": (256,), "W2": (256, 256), "b2": (256,), "W3": (K, 256),
              "b3": (K,)}
    out, o = {}, 0
    for k in PARAM_NAMES:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + n]).reshape(shapes[k])
        o += n
    return out


class MLP:
    """Proposal network handle (float32 parameters on the device)."""

    def __init__(self, K: int, params, max_batch: int = 4096):
        v = params if isinstance(params, np.ndarray) else flatten_params(params)
        v = np.ascontiguousarray(v, dtype=np.float32)
        if v.size != lib().fepll_mlp_param_count(K):
            raise ValueError("parameter vector has the wrong length")
        h = c_void_p()
        _check(lib().fepll_mlp_create(K, v.ctypes.data, int(max_batch), ctypes.byref(h)))
        self._h = h
        self.K = K
        self.max_batch = max_batch

    def close(self):
        if getattr(self, "_h", None):
            lib().fepll_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        v = np.empty(lib().fepll_mlp_param_count(self.K), np.float32)
        _check(lib().fepll_mlp_get_params(self._h, v.ctypes.data))
        return v

    def forward(self, X):
        import torch
        n = X.shape[0]
        out = torch.empty((n, self.K), dtype=torch.float32, device=X.device)
        _check(lib().fepll_mlp_forward(self._h, X.data_ptr(), n, out.data_ptr(), _stream_of(X)))
        return out

    def loss_grad(self, X, y):
        import torch
        g = torch.empty(lib().fepll_mlp_param_count(self.K), dtype=torch.float32,
                        device=X.device)
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
        _check(lib().fepll_mlp_loss_grad(self._h, X.data_ptr(), y.data_ptr(), X.shape[0],
                                         g.data_ptr(), loss.data_ptr(), _stream_of(X)))
        return loss, g

    def train_step(self, X, y, rows=None, n=None, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                   weight_decay=1e-4, loss=None):
        hp = AdamW(lr, beta1, beta2, eps, weight_decay)
        if n is None:
            n = rows.shape[0] if rows is not None else X.shape[0]
        _check(lib().fepll_mlp_train_step(self._h, X.data_ptr(), y.data_ptr(),
                                          rows.data_ptr() if rows is not None else None, int(n),
                                          ctypes.byref(hp),
                                          loss.data_ptr() if loss is not None else None,
                                          _stream_of(X)))

    def serialize(self) -> bytes:
        nb = ctypes.c_size_t()
        _check(lib().fepll_mlp_serialize(self._h, None, 0, ctypes.byref(nb)))
        buf = ctypes.create_string_buffer(nb.value)
        _check(lib().fepll_mlp_serialize(self._h, buf, nb.value, ctypes.byref(nb)))
        return buf.raw[:nb.value]
