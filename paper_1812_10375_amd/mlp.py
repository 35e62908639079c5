"""Python binding of the surrogate network library (``include/lbm_mlp.h``).

Argument marshalling only: forward and backward passes and the Adam update run in the
BF16 matrix-core kernels of ``liblbm_hip.so``.  Torch provides device memory and the
stream.  Host arrays are float32 in the layout of lbm_mlp_params().
"""
import ctypes as C

import numpy as np

from .lbm import LbmError, library

_bound = False


def _lib():
    global _bound
    L = library()
    if not _bound:
        vp = C.c_void_p
        fp = C.POINTER(C.c_float)
        L.lbm_mlp_params.restype = C.c_size_t
        L.lbm_mlp_params.argtypes = []
        L.lbm_mlp_workspace_bytes.restype = C.c_size_t
        L.lbm_mlp_workspace_bytes.argtypes = [C.c_int, C.c_int]
        L.lbm_mlp_init.restype = C.c_int
        L.lbm_mlp_init.argtypes = [C.c_int, C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)]
        for name in ("lbm_mlp_set_params", "lbm_mlp_get_params", "lbm_mlp_get_grads"):
            getattr(L, name).restype = C.c_int
            getattr(L, name).argtypes = [vp, fp]
        L.lbm_mlp_forward.restype = C.c_int
        L.lbm_mlp_forward.argtypes = [vp, vp, C.c_int, vp]
        L.lbm_mlp_forward_noalloc.restype = C.c_int
        L.lbm_mlp_forward_noalloc.argtypes = [vp, vp, C.c_int, vp]
        L.lbm_mlp_backward.restype = C.c_int
        L.lbm_mlp_backward.argtypes = [vp, vp, vp, C.c_int, C.c_int, vp]
        L.lbm_mlp_adam.restype = C.c_int
        L.lbm_mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
        L.lbm_mlp_destroy.restype = C.c_int
        L.lbm_mlp_destroy.argtypes = [vp]
        _bound = True
    return L


NOALLOC_MAX_ROWS = 8192  # LBM_MLP_NOALLOC_MAX_ROWS of include/lbm_mlp.h


def n_params():
    return int(_lib().lbm_mlp_params())


class MLPEnsemble:
    """An ensemble of surrogate networks on the GPU (BF16 matrix-core kernels)."""

    def __init__(self, members, max_batch, params=None, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the surrogate library needs a GPU")
        L = _lib()
        self.torch = torch
        self.members, self.max_batch = int(members), int(max_batch)
        self.device = torch.device("cuda") if device is None else torch.device(device)
        nbytes = L.lbm_mlp_workspace_bytes(self.members, self.max_batch)
        if nbytes == 0:
            raise LbmError(-1, "lbm_mlp_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.loss = torch.zeros(self.members, dtype=torch.float32, device=self.device)
        h = C.c_void_p()
        rc = L.lbm_mlp_init(self.members, self.max_batch, C.c_void_p(self.ws.data_ptr()), nbytes,
                            C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_init")
        self.h = h
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "h", None):
            _lib().lbm_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _host(self, arr):
        a = np.ascontiguousarray(np.asarray(arr, dtype=np.float32).reshape(self.members, n_params()))
        return a, a.ctypes.data_as(C.POINTER(C.c_float))

    def set_params(self, params):
        a, p = self._host(params)
        rc = _lib().lbm_mlp_set_params(self.h, p)
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_set_params")

    def params(self):
        a, p = self._host(np.zeros((self.members, n_params())))
        rc = _lib().lbm_mlp_get_params(self.h, p)
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_get_params")
        return a.astype(np.float64)

    def grads(self):
        a, p = self._host(np.zeros((self.members, n_params())))
        rc = _lib().lbm_mlp_get_grads(self.h, p)
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_get_grads")
        return a.astype(np.float64)

    def _dev(self, x, cols, allow_members=False):
        t = self.torch.as_tensor(np.asarray(x, dtype=np.float32)) if not self.torch.is_tensor(x) else x
        t = t.to(device=self.device, dtype=self.torch.float32).contiguous()
        ok = (t.dim() == 2 and t.shape[1] == cols) or (
            allow_members and t.dim() == 3 and t.shape[0] == self.members and t.shape[2] == cols)
        if not ok:
            raise ValueError("expected a [B][%d] array%s" % (cols, " or [members][B][%d]" % cols if allow_members else ""))
        return t

    def forward(self, x):
        """Outputs of every member, a device tensor [members][B][2]."""
        xt = self._dev(x, 4)
        B = xt.shape[0]
        y = self.torch.empty((self.members, B, 2), dtype=self.torch.float32, device=self.device)
        rc = _lib().lbm_mlp_forward(self.h, C.c_void_p(xt.data_ptr()), B, C.c_void_p(y.data_ptr()))
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_forward")
        self._keep = xt
        return y

    def forward_noalloc(self, x, y=None):
        """The same outputs through the allocation-free entry point (activations in the
        library's fixed device array; members * B <= NOALLOC_MAX_ROWS).  `y`, if given,
        is a device tensor [members][B][2] to write into."""
        xt = self._dev(x, 4)
        B = xt.shape[0]
        if y is None:
            y = self.torch.empty((self.members, B, 2), dtype=self.torch.float32, device=self.device)
        rc = _lib().lbm_mlp_forward_noalloc(self.h, C.c_void_p(xt.data_ptr()), B, C.c_void_p(y.data_ptr()))
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_forward_noalloc")
        self._keep = xt
        return y

    def backward(self, x, t):
        """Loss and gradients of every member on (x, t): arrays [B][4], [B][2] shared by
        all members, or [members][B][4], [members][B][2] with one batch per member.
        Returns the device loss tensor."""
        xt, tt = self._dev(x, 4, True), self._dev(t, 2, True)
        per = int(xt.dim() == 3)
        if tt.dim() != xt.dim() or tt.shape[-2] != xt.shape[-2]:
            raise ValueError("inputs and targets do not match")
        B = xt.shape[-2]
        rc = _lib().lbm_mlp_backward(self.h, C.c_void_p(xt.data_ptr()), C.c_void_p(tt.data_ptr()), B, per,
                                     C.c_void_p(self.loss.data_ptr()))
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_backward")
        self._keep = (xt, tt)
        return self.loss

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        rc = _lib().lbm_mlp_adam(self.h, float(lr), float(beta1), float(beta2), float(eps))
        if rc != 0:
            raise LbmError(rc, "lbm_mlp_adam")

    def train_step(self, x, t, lr):
        loss = self.backward(x, t)
        self.adam(lr)
        return loss
