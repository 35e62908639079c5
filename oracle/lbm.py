"""ctypes binding of the C oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE (see the package docstring).  ``OracleSim`` takes a scenario
dictionary (the same one the GPU binding takes) and runs the FP64 oracle on it.
"""
import ctypes as C
import os

import numpy as np

from .build import build_oracle, library_path

TOP_BC = {"wall": 0, "const_pressure": 1, "convective": 2}
TBC = {"dirichlet": 0, "flux": 1, "zero_grad": 2}
FLAG_BITS = {"freeze_eos_T": 1, "no_advection": 2, "no_latent": 4, "diff_isotropic": 8,
             "sigma_plain": 16}
FIELDS = {"f": 0, "rho": 1, "ux": 2, "uy": 3, "T": 4, "psi": 5, "Fx": 6, "Fy": 7, "Fmx": 8,
          "Fmy": 9, "Gw": 10}
ERR_BITS = {"rho": 1, "covolume": 2, "radicand": 4, "nonfinite": 8}


class OrcParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("heater_rows", C.c_int32),
                ("n_sub", C.c_int32), ("top_bc", C.c_int32), ("bottom_tbc", C.c_int32),
                ("top_tbc", C.c_int32), ("flags", C.c_uint32)] + [
        (n, C.c_double) for n in (
            "a", "b", "R", "omega", "T_sat", "G", "sigma", "tau_l", "tau_v", "s_e", "s_zeta",
            "s_q", "rho_l", "rho_v", "cv", "k", "rho_w", "cv_w", "lambda_w", "g", "T_bottom",
            "T_top", "q_bottom", "Gw0", "Gw_top")] + [
        ("n_sites", C.c_int32), ("site_xc", C.POINTER(C.c_double)),
        ("site_width", C.POINTER(C.c_double)), ("site_gmin", C.POINTER(C.c_double))]


class OrcObs(C.Structure):
    _fields_ = [("step", C.c_int64)] + [
        (n, C.c_double) for n in (
            "mass", "energy", "rho_ave", "q_bottom", "q_bottom_mean", "q_bottom_var",
            "q_surface", "Q_bottom_cum", "Q_top_cum", "Q_surface_cum", "dE_cum",
            "max_speed")] + [("error_flags", C.c_int32), ("first_bad_step", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(library_path()):
            build_oracle()
        L = C.CDLL(library_path())
        P = C.POINTER(OrcParams)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [P, dp, dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_step.restype = C.c_int
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_observe.argtypes = [C.c_void_p, C.POINTER(OrcObs)]
        L.orc_field.restype = dp
        L.orc_field.argtypes = [C.c_void_p, C.c_int]
        L.orc_field_len.restype = C.c_int64
        L.orc_field_len.argtypes = [C.c_void_p, C.c_int]
        for name in ("orc_eos_p", "orc_psi", "orc_dpdT"):
            getattr(L, name).restype = C.c_double
            getattr(L, name).argtypes = [P, C.c_double, C.c_double]
        L.orc_Tc.restype = C.c_double
        L.orc_Tc.argtypes = [P]
        L.orc_feq.argtypes = [C.c_double, C.c_double, C.c_double, dp]
        L.orc_collide_node.argtypes = [P, dp] + [C.c_double] * 5 + [dp, dp, dp]
        for name in ("orc_moments", "orc_forces", "orc_energy_update"):
            getattr(L, name).argtypes = [C.c_void_p]
        L.orc_energy_rhs.argtypes = [C.c_void_p, dp, dp, dp]
        _lib = L
    return _lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(sc):
    """Marshal a scenario dictionary into the oracle's parameter struct."""
    p = OrcParams()
    p.nx, p.ny, p.heater_rows = sc["nx"], sc["ny"], sc["heater_rows"]
    p.n_sub = sc.get("n_sub", 1)
    p.top_bc = TOP_BC[sc["top_bc"]]
    p.bottom_tbc = TBC[sc["bottom_tbc"]]
    p.top_tbc = TBC[sc["top_tbc"]]
    p.flags = sum(FLAG_BITS[f] for f in sc.get("flags", ()))
    for n in ("a", "b", "R", "omega", "T_sat", "G", "sigma", "tau_l", "tau_v", "s_e", "s_zeta",
              "s_q", "rho_l", "rho_v", "cv", "k", "rho_w", "cv_w", "lambda_w", "g", "T_bottom",
              "T_top", "q_bottom", "Gw0", "Gw_top"):
        setattr(p, n, float(sc[n]))
    sites = np.asarray(sc.get("sites", np.zeros((0, 3))), dtype=np.float64).reshape(-1, 3)
    keep = [np.ascontiguousarray(sites[:, k]) for k in range(3)]
    p.n_sites = sites.shape[0]
    p.site_xc, p.site_width, p.site_gmin = (_dptr(k) for k in keep)
    return p, keep


class OracleSim:
    """FP64 oracle run of one scenario."""

    def __init__(self, sc, rho0=None, T0=None):
        self.sc = sc
        self.p, self._keep = make_params(sc)
        rho0 = np.ascontiguousarray(sc["rho0"] if rho0 is None else rho0, dtype=np.float64)
        T0 = np.ascontiguousarray(sc["T0"] if T0 is None else T0, dtype=np.float64)
        nx, ny, nh = sc["nx"], sc["ny"], sc["heater_rows"]
        assert rho0.shape == (ny, nx) and T0.shape == (nh + ny, nx)
        self.h = lib().orc_create(C.byref(self.p), _dptr(rho0), _dptr(T0))
        if not self.h:
            raise ValueError("oracle rejected the scenario")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def step(self, n=1):
        return lib().orc_step(self.h, int(n))

    def observe(self):
        o = OrcObs()
        lib().orc_observe(self.h, C.byref(o))
        return {k: getattr(o, k) for k, _ in OrcObs._fields_}

    def _view(self, name):
        f = FIELDS[name]
        n = lib().orc_field_len(self.h, f)
        ptr = lib().orc_field(self.h, f)
        return np.ctypeslib.as_array(ptr, shape=(n,))

    def _shape(self, name):
        nx, ny, nh = self.sc["nx"], self.sc["ny"], self.sc["heater_rows"]
        if name == "f":
            return (9, ny, nx)
        if name == "T":
            return (nh + ny, nx)
        if name == "Gw":
            return (nx,)
        return (ny, nx)

    def field(self, name):
        """Copy of an internal field (see lbm_oracle.h for meaning and layout)."""
        return self._view(name).reshape(self._shape(name)).copy()

    def set_field(self, name, values):
        v = self._view(name)
        v[:] = np.asarray(values, dtype=np.float64).reshape(-1)

    # building blocks -------------------------------------------------------
    def moments(self):
        lib().orc_moments(self.h)

    def forces(self):
        lib().orc_forces(self.h)

    def energy_update(self):
        lib().orc_energy_update(self.h)

    def energy_rhs(self, Y):
        Y = np.ascontiguousarray(Y, dtype=np.float64)
        K = np.zeros_like(Y)
        flux = np.zeros(3)
        lib().orc_energy_rhs(self.h, _dptr(Y), _dptr(K), _dptr(flux))
        return K, flux


def eos_p(sc, rho, T):
    p, keep = make_params(sc)
    return lib().orc_eos_p(C.byref(p), float(rho), float(T))


def psi(sc, rho, T):
    p, keep = make_params(sc)
    return lib().orc_psi(C.byref(p), float(rho), float(T))


def dpdT(sc, rho, T):
    p, keep = make_params(sc)
    return lib().orc_dpdT(C.byref(p), float(rho), float(T))


def Tc(sc):
    p, keep = make_params(sc)
    return lib().orc_Tc(C.byref(p))


def feq(rho, ux, uy):
    out = np.zeros(9)
    lib().orc_feq(float(rho), float(ux), float(uy), _dptr(out))
    return out


def collide_node(sc, f, Fx, Fy, Fmx, Fmy, psi_c):
    p, keep = make_params(sc)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros(9)
    ux = C.c_double()
    uy = C.c_double()
    lib().orc_collide_node(C.byref(p), _dptr(f), Fx, Fy, Fmx, Fmy, psi_c, _dptr(out),
                           C.byref(ux), C.byref(uy))
    return out, ux.value, uy.value
