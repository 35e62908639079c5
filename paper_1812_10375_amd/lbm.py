"""Python binding of the gfx950 library (``include/lbm_api.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``liblbm_hip.so``.  PyTorch provides the device workspace and the stream.  There is
no CPU fallback: without the built library (or without a GPU) construction fails.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_hip.so")

F32, F64 = 0, 1
TOP_BC = {"wall": 0, "const_pressure": 1, "convective": 2}
TBC = {"dirichlet": 0, "flux": 1, "zero_grad": 2}
FLAG_BITS = {"freeze_eos_T": 1, "no_advection": 2, "no_latent": 4, "diff_isotropic": 8,
             "two_launches": 32, "one_launch": 64}
FIELDS = {"f": 0, "rho": 1, "ux": 2, "uy": 3, "T": 4, "Gw": 10, "state": 11}
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP",
          -4: "LBM_ENONFINITE", -5: "LBM_ESTATE"}
ABI_VERSION = 2


class LbmConfig(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("abi_version", C.c_uint32),
                ("nx", C.c_int32), ("ny", C.c_int32), ("heater_rows", C.c_int32), ("n_sub", C.c_int32),
                ("precision", C.c_int32), ("top_bc", C.c_int32), ("bottom_tbc", C.c_int32),
                ("top_tbc", C.c_int32), ("flags", C.c_uint32), ("tile_rows", C.c_int32)] + [
        (n, C.c_double) for n in (
            "a", "b", "R", "omega", "T_sat", "G", "sigma", "tau_l", "tau_v", "s_e", "s_zeta", "s_q",
            "rho_l", "rho_v", "cv", "k", "rho_w", "cv_w", "lambda_w", "g", "T_bottom", "T_top",
            "q_bottom", "Gw0", "Gw_top")] + [
        ("n_sites", C.c_int32), ("site_xc", C.POINTER(C.c_double)),
        ("site_width", C.POINTER(C.c_double)), ("site_gmin", C.POINTER(C.c_double))]


class LbmObs(C.Structure):
    _fields_ = [("step", C.c_int64)] + [
        (n, C.c_double) for n in (
            "mass", "energy", "rho_ave", "q_bottom", "q_bottom_mean", "q_bottom_var", "q_surface",
            "Q_bottom_cum", "Q_top_cum", "Q_surface_cum", "dE_cum", "max_speed")] + [
        ("error_flags", C.c_int32), ("first_bad_step", C.c_int64)]


class LbmError(RuntimeError):
    def __init__(self, status, what):
        super().__init__("%s failed: %s (%d)" % (what, STATUS.get(status, "?"), status))
        self.status = status


_lib = None


def library():
    """The loaded C-ABI library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblbm_hip.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        cfgp = C.POINTER(LbmConfig)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.lbm_workspace_bytes.restype = C.c_size_t
        L.lbm_workspace_bytes.argtypes = [cfgp]
        L.lbm_init.restype = C.c_int
        L.lbm_init.argtypes = [cfgp, vp, C.c_size_t, vp, dp, dp, C.POINTER(vp)]
        L.lbm_step.restype = C.c_int
        L.lbm_step.argtypes = [vp, C.c_int64]
        L.lbm_observe.restype = C.c_int
        L.lbm_observe.argtypes = [vp, C.POINTER(LbmObs)]
        L.lbm_read_field.restype = C.c_int
        L.lbm_read_field.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
        L.lbm_write_field.restype = C.c_int
        L.lbm_write_field.argtypes = [vp, C.c_int, vp, C.c_size_t, C.c_int]
        L.lbm_field_bytes.restype = C.c_size_t
        L.lbm_field_bytes.argtypes = [vp, C.c_int]
        L.lbm_destroy.restype = C.c_int
        L.lbm_destroy.argtypes = [vp]
        L.lbm_set_stream.restype = C.c_int
        L.lbm_set_stream.argtypes = [vp, vp]
        L.lbm_set_kernel_timing.restype = C.c_int
        L.lbm_set_kernel_timing.argtypes = [vp, C.c_int]
        L.lbm_kernel_times.restype = C.c_int
        L.lbm_kernel_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.lbm_strerror.restype = C.c_char_p
        L.lbm_strerror.argtypes = [C.c_int]
        bp = C.c_void_p
        dpp = C.POINTER(C.POINTER(C.c_double))
        L.lbm_batch_workspace_bytes.restype = C.c_size_t
        L.lbm_batch_workspace_bytes.argtypes = [cfgp, C.c_int]
        L.lbm_batch_init.restype = C.c_int
        L.lbm_batch_init.argtypes = [cfgp, C.c_int, vp, C.c_size_t, vp, dpp, dpp, C.POINTER(bp)]
        L.lbm_batch_step.restype = C.c_int
        L.lbm_batch_step.argtypes = [bp, C.c_int64]
        L.lbm_batch_set_stream.restype = C.c_int
        L.lbm_batch_set_stream.argtypes = [bp, vp]
        L.lbm_batch_observe.restype = C.c_int
        L.lbm_batch_observe.argtypes = [bp, C.POINTER(LbmObs)]
        L.lbm_batch_read_field.restype = C.c_int
        L.lbm_batch_read_field.argtypes = [bp, C.c_int, C.c_int, vp, C.c_size_t, C.c_int]
        L.lbm_batch_write_field.restype = C.c_int
        L.lbm_batch_write_field.argtypes = [bp, C.c_int, C.c_int, vp, C.c_size_t, C.c_int]
        L.lbm_batch_destroy.restype = C.c_int
        L.lbm_batch_destroy.argtypes = [bp]
        L.lbm_autotune_tile_rows.restype = C.c_int
        L.lbm_autotune_tile_rows.argtypes = [cfgp, C.c_int, vp, C.c_size_t, vp, dpp, dpp, C.c_int,
                                             C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.lbm_autotune.restype = C.c_int
        L.lbm_autotune.argtypes = [cfgp, C.c_int, vp, C.c_size_t, vp, dpp, dpp, C.c_int,
                                   C.POINTER(C.c_int32), C.POINTER(C.c_uint32), C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(sc):
    """Marshal a scenario dictionary into lbm_config (returns it and the arrays it points to)."""
    c = LbmConfig()
    c.struct_size = C.sizeof(LbmConfig)
    c.abi_version = ABI_VERSION
    c.nx, c.ny, c.heater_rows = sc["nx"], sc["ny"], sc["heater_rows"]
    c.n_sub = sc.get("n_sub", 1)
    c.precision = F64 if sc.get("precision", "f64") == "f64" else F32
    c.top_bc = TOP_BC[sc["top_bc"]]
    c.bottom_tbc = TBC[sc["bottom_tbc"]]
    c.top_tbc = TBC[sc["top_tbc"]]
    c.flags = sum(FLAG_BITS[f] for f in sc.get("flags", ()))
    c.tile_rows = int(sc.get("tile_rows", 0))
    for n in ("a", "b", "R", "omega", "T_sat", "G", "sigma", "tau_l", "tau_v", "s_e", "s_zeta",
              "s_q", "rho_l", "rho_v", "cv", "k", "rho_w", "cv_w", "lambda_w", "g", "T_bottom",
              "T_top", "q_bottom", "Gw0", "Gw_top"):
        setattr(c, n, float(sc[n]))
    sites = np.asarray(sc.get("sites", np.zeros((0, 3))), dtype=np.float64).reshape(-1, 3)
    keep = [np.ascontiguousarray(sites[:, k]) for k in range(3)]
    c.n_sites = sites.shape[0]
    c.site_xc, c.site_width, c.site_gmin = (_dptr(k) for k in keep)
    return c, keep


def workspace_bytes(sc):
    c, keep = make_config(sc)
    return library().lbm_workspace_bytes(C.byref(c))


class Lattice:
    """One domain on the current GPU, advanced by the library's kernels."""

    def __init__(self, sc, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the hybrid LB library needs a GPU")
        L = library()
        self.sc = sc
        self.torch = torch
        self.device = torch.device("cuda") if device is None else torch.device(device)
        self.cfg, self._keep = make_config(sc)
        self.dtype = np.float64 if self.cfg.precision == F64 else np.float32
        nbytes = L.lbm_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise LbmError(-1, "lbm_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        rho0 = np.ascontiguousarray(sc["rho0"], dtype=np.float64)
        T0 = np.ascontiguousarray(sc["T0"], dtype=np.float64)
        nx, ny, nh = sc["nx"], sc["ny"], sc["heater_rows"]
        if rho0.shape != (ny, nx) or T0.shape != (nh + ny, nx):
            raise ValueError("initial field shapes do not match the lattice")
        h = C.c_void_p()
        rc = L.lbm_init(C.byref(self.cfg), C.c_void_p(self.ws.data_ptr()), nbytes,
                        C.c_void_p(self.stream.cuda_stream), _dptr(rho0), _dptr(T0), C.byref(h))
        if rc != 0:
            raise LbmError(rc, "lbm_init")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            library().lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        rc = library().lbm_step(self.h, int(n))
        if rc != 0:
            raise LbmError(rc, "lbm_step")

    def observe(self, check=True):
        o = LbmObs()
        rc = library().lbm_observe(self.h, C.byref(o))
        d = {k: getattr(o, k) for k, _ in LbmObs._fields_}
        d["status"] = rc
        if check and rc != 0:
            raise LbmError(rc, "lbm_observe")
        return d

    def set_stream(self, stream):
        """Enqueue later work on `stream` (a torch stream), e.g. a graph-capture stream."""
        rc = library().lbm_set_stream(self.h, C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise LbmError(rc, "lbm_set_stream")
        self.stream = stream

    def set_kernel_timing(self, on):
        rc = library().lbm_set_kernel_timing(self.h, int(bool(on)))
        if rc != 0:
            raise LbmError(rc, "lbm_set_kernel_timing")

    def kernel_times(self):
        """{'collide': (ms, launches), 'energy': (ms, launches)} since the last read."""
        cm, em = C.c_double(), C.c_double()
        cn, en = C.c_int64(), C.c_int64()
        rc = library().lbm_kernel_times(self.h, C.byref(cm), C.byref(cn), C.byref(em), C.byref(en))
        if rc != 0:
            raise LbmError(rc, "lbm_kernel_times")
        return {"collide": (cm.value, cn.value), "energy": (em.value, en.value)}

    def _shape(self, name):
        nx, ny, nh = self.sc["nx"], self.sc["ny"], self.sc["heater_rows"]
        return {"f": (9, ny, nx), "T": (nh + ny, nx), "Gw": (nx,)}.get(name, (ny, nx))

    def read(self, name):
        """Host copy of a field, as float64."""
        out = np.empty(self._shape(name), dtype=self.dtype)
        rc = library().lbm_read_field(self.h, FIELDS[name], out.ctypes.data_as(C.c_void_p),
                                      out.nbytes, 0)
        if rc != 0:
            raise LbmError(rc, "lbm_read_field")
        return out.astype(np.float64)

    def write(self, name, values):
        arr = np.ascontiguousarray(np.asarray(values).reshape(self._shape(name)), dtype=self.dtype)
        rc = library().lbm_write_field(self.h, FIELDS[name], arr.ctypes.data_as(C.c_void_p),
                                       arr.nbytes, 0)
        if rc != 0:
            raise LbmError(rc, "lbm_write_field")

    def read_state(self):
        """The run state beyond the fields (LBM_FIELD_STATE) as raw bytes."""
        n = library().lbm_field_bytes(self.h, FIELDS["state"])
        out = np.zeros(n, dtype=np.uint8)
        rc = library().lbm_read_field(self.h, FIELDS["state"], out.ctypes.data_as(C.c_void_p), n, 0)
        if rc != 0:
            raise LbmError(rc, "lbm_read_field(state)")
        return out

    def write_state(self, rec):
        rec = np.ascontiguousarray(rec, dtype=np.uint8)
        rc = library().lbm_write_field(self.h, FIELDS["state"], rec.ctypes.data_as(C.c_void_p), rec.nbytes, 0)
        if rc != 0:
            raise LbmError(rc, "lbm_write_field(state)")

    def checkpoint(self):
        """Everything a run continues from: populations, temperature and run state, in
        the field precision (a dict of host arrays)."""
        out = {}
        for name in ("f", "T"):
            arr = np.empty(self._shape(name), dtype=self.dtype)
            rc = library().lbm_read_field(self.h, FIELDS[name], arr.ctypes.data_as(C.c_void_p), arr.nbytes, 0)
            if rc != 0:
                raise LbmError(rc, "lbm_read_field")
            out[name] = arr
        out["state"] = self.read_state()
        return out

    def restore(self, ckpt):
        """Continue from a checkpoint of a run of the same configuration."""
        self.write("f", ckpt["f"])
        self.write("T", ckpt["T"])
        self.write_state(ckpt["state"])


def _shape_of(sc, name):
    nx, ny, nh = sc["nx"], sc["ny"], sc["heater_rows"]
    return {"f": (9, ny, nx), "T": (nh + ny, nx), "Gw": (nx,)}.get(name, (ny, nx))


class _BatchInputs:
    """Marshalled configurations and initial fields of a list of scenarios."""

    def __init__(self, scs):
        n = len(scs)
        self.n = n
        self.cfgs = (LbmConfig * n)()
        self.keep = []
        self.fields = []
        for i, sc in enumerate(scs):
            c, keep = make_config(sc)
            self.cfgs[i] = c
            self.keep.append(keep)
            nx, ny, nh = sc["nx"], sc["ny"], sc["heater_rows"]
            rho0 = np.ascontiguousarray(sc["rho0"], dtype=np.float64)
            T0 = np.ascontiguousarray(sc["T0"], dtype=np.float64)
            if rho0.shape != (ny, nx) or T0.shape != (nh + ny, nx):
                raise ValueError("initial field shapes do not match the lattice of domain %d" % i)
            self.fields.append((rho0, T0))
        DP = C.POINTER(C.c_double)
        self.rho0 = (DP * n)(*[_dptr(r) for r, _ in self.fields])
        self.T0 = (DP * n)(*[_dptr(t) for _, t in self.fields])

    def workspace_bytes(self):
        return library().lbm_batch_workspace_bytes(self.cfgs, self.n)


class BatchLattice:
    """Independent domains advanced together by the batched kernels (one collide and
    n_sub energy launches per step for the whole batch)."""

    def __init__(self, scs, device=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the hybrid LB library needs a GPU")
        L = library()
        self.scs = list(scs)
        self.inp = _BatchInputs(self.scs)
        self.device = torch.device("cuda") if device is None else torch.device(device)
        nbytes = self.inp.workspace_bytes()
        if nbytes == 0:
            raise LbmError(-1, "lbm_batch_workspace_bytes")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        self.dtype = np.float64 if self.inp.cfgs[0].precision == F64 else np.float32
        h = C.c_void_p()
        rc = L.lbm_batch_init(self.inp.cfgs, self.inp.n, C.c_void_p(self.ws.data_ptr()), nbytes,
                              C.c_void_p(self.stream.cuda_stream), self.inp.rho0, self.inp.T0, C.byref(h))
        if rc != 0:
            raise LbmError(rc, "lbm_batch_init")
        self.h = h

    def __len__(self):
        return self.inp.n

    def close(self):
        if getattr(self, "h", None):
            library().lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n=1):
        rc = library().lbm_batch_step(self.h, int(n))
        if rc != 0:
            raise LbmError(rc, "lbm_batch_step")

    def set_stream(self, stream):
        rc = library().lbm_batch_set_stream(self.h, C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise LbmError(rc, "lbm_batch_set_stream")
        self.stream = stream

    def observe(self, check=True):
        """List of per-domain observation dictionaries."""
        obs = (LbmObs * self.inp.n)()
        rc = library().lbm_batch_observe(self.h, obs)
        if check and rc != 0:
            raise LbmError(rc, "lbm_batch_observe")
        out = []
        for o in obs:
            d = {k: getattr(o, k) for k, _ in LbmObs._fields_}
            d["status"] = rc
            out.append(d)
        return out

    def read(self, i, name):
        out = np.empty(_shape_of(self.scs[i], name), dtype=self.dtype)
        rc = library().lbm_batch_read_field(self.h, int(i), FIELDS[name], out.ctypes.data_as(C.c_void_p),
                                            out.nbytes, 0)
        if rc != 0:
            raise LbmError(rc, "lbm_batch_read_field")
        return out.astype(np.float64)

    def write(self, i, name, values):
        arr = np.ascontiguousarray(np.asarray(values).reshape(_shape_of(self.scs[i], name)), dtype=self.dtype)
        rc = library().lbm_batch_write_field(self.h, int(i), FIELDS[name], arr.ctypes.data_as(C.c_void_p),
                                             arr.nbytes, 0)
        if rc != 0:
            raise LbmError(rc, "lbm_batch_write_field")


def autotune_tile_rows(scs, steps=20, device=None, stream=None):
    """Fastest energy tile height for this batch of scenarios (cached per process by the
    library): returns (tile_rows, ms per step)."""
    import torch
    inp = _BatchInputs(scs)
    nbytes = inp.workspace_bytes()
    if nbytes == 0:
        raise LbmError(-1, "lbm_batch_workspace_bytes")
    dev = torch.device("cuda") if device is None else torch.device(device)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream(dev) if stream is None else stream
    rows, ms = C.c_int(), C.c_double()
    rc = library().lbm_autotune_tile_rows(inp.cfgs, inp.n, C.c_void_p(ws.data_ptr()), nbytes,
                                          C.c_void_p(st.cuda_stream), inp.rho0, inp.T0, int(steps),
                                          C.byref(rows), C.byref(ms))
    if rc != 0:
        raise LbmError(rc, "lbm_autotune_tile_rows")
    return rows.value, ms.value


def autotune(scs, steps=20, device=None, stream=None):
    """Launch shape for these scenarios (a batch, or one domain on its own path), cached
    per process by the library: returns (scenarios with the chosen tile_rows and launch
    mode, ms per step)."""
    import torch
    inp = _BatchInputs(scs)
    nbytes = inp.workspace_bytes()
    if nbytes == 0:
        raise LbmError(-1, "lbm_batch_workspace_bytes")
    dev = torch.device("cuda") if device is None else torch.device(device)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream(dev) if stream is None else stream
    rows, flags, ms = (C.c_int32 * inp.n)(), (C.c_uint32 * inp.n)(), C.c_double()
    rc = library().lbm_autotune(inp.cfgs, inp.n, C.c_void_p(ws.data_ptr()), nbytes, C.c_void_p(st.cuda_stream),
                                inp.rho0, inp.T0, int(steps), rows, flags, C.byref(ms))
    if rc != 0:
        raise LbmError(rc, "lbm_autotune")
    out = []
    for sc, r, f in zip(scs, rows, flags):
        names = tuple(k for k, bit in FLAG_BITS.items() if f & bit)
        out.append(dict(sc, tile_rows=int(r), flags=names))
    return out, ms.value
