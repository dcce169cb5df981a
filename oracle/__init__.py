"""ctypes binding of the FP64 CPU oracle (``oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and by
the CPU-baseline leg of the benchmark. The product library never imports it.

All field arrays are float64, C-contiguous, shape (C, Ny + 4, Nx + 4) with the
width-2 halo; helpers copy their inputs so callers' arrays are not modified
unless a function says so.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

THEORIES = {"abelian_higgs": 0, "chiral_magnet": 1, "toy_harmonic": 2, "toy_offset": 3, "baby_skyrme": 4,
            # chiral magnet with a second DMI coefficient and demagnetisation:
            # params {J, D, K, B, Dy, mu_d} (Dy = D bulk, -D Heusler; mu_d = 0: no demagnetisation)
            "chiral_magnet_ext": 5,
            # rotating trapped BEC in trap units, params {g, Omega, N}; the flow holds
            # the atom number N = h^2 sum |psi|^2 fixed
            "bec": 6}
COURANT = 0.5  # dt = C * h with the default C of Sec. 3.1
GRAD_EXACT = 0  # G = h^-2 dE_h/dphi
GRAD_EL = 1     # continuum Euler-Lagrange expression evaluated with eq. (1)-(2)
# integrators of the flow: classical RK4, velocity Verlet, gradient flow
SCHEMES = {"rk4": 0, "vv": 1, "gf": 2}


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math, one thread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.or_components.argtypes = [i]
        L.or_components.restype = i
        L.or_deriv_at.argtypes = [dp, i, i, d, i, i, i, i, i]
        L.or_deriv_at.restype = d
        L.or_energy.argtypes = [i, i, i, d, dp, dp]
        L.or_energy.restype = d
        L.or_energy_density.argtypes = [i, i, i, d, dp, dp, dp]
        L.or_energy_complex.argtypes = [i, i, i, d, dp, dp, dp, dp]
        L.or_gradient.argtypes = [i, i, i, i, d, dp, dp, dp]
        L.or_acceleration.argtypes = [i, i, i, i, d, dp, dp, dp]
        L.or_flow.argtypes = [i, i, i, i, d, dp, d, dp, dp, dp, i, ctypes.POINTER(ctypes.c_long)]
        L.or_minimise.argtypes = [i, i, i, i, d, dp, d, dp, dp, d, d, i, ctypes.c_long, dp]
        L.or_flow_scheme.argtypes = [i, i, i, i, i, d, dp, d, dp, dp, dp, i, ctypes.POINTER(ctypes.c_long)]
        L.or_minimise_scheme.argtypes = [i, i, i, i, i, d, dp, d, dp, dp, d, d, i, ctypes.c_long, dp]
        L.or_observables_ah.argtypes = [i, i, d, dp, dp, dp]
        L.or_observables_cm.argtypes = [i, i, d, dp, dp, dp]
        L.or_observables_unit.argtypes = [i, i, i, d, dp, dp, dp]
        L.or_observables_bec.argtypes = [i, i, d, dp, dp, dp]
        L.or_poisson.argtypes = [i, i, d, dp, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def _dims(phi: np.ndarray):
    C, H, W = phi.shape
    return W - 4, H - 4


def _tid(theory) -> int:
    return THEORIES[theory] if isinstance(theory, str) else int(theory)


def deriv_at(phi, h, c, j, i, axis) -> float:
    phi = _arr(phi)
    Nx, Ny = _dims(phi)
    return lib().or_deriv_at(_p(phi), Nx, Ny, h, phi.shape[0], c, j, i, axis)


def energy(theory, phi, h, params) -> float:
    phi, p = _arr(phi), _arr(params)
    Nx, Ny = _dims(phi)
    return lib().or_energy(_tid(theory), Nx, Ny, h, _p(p), _p(phi))


def energy_density(theory, phi, h, params) -> np.ndarray:
    phi, p = _arr(phi), _arr(params)
    Nx, Ny = _dims(phi)
    out = np.zeros((Ny, Nx))
    lib().or_energy_density(_tid(theory), Nx, Ny, h, _p(p), _p(phi), _p(out))
    return out


def energy_complex(theory, re, im, h, params) -> complex:
    re, im, p = _arr(re), _arr(im), _arr(params)
    Nx, Ny = _dims(re)
    out = np.zeros(2)
    lib().or_energy_complex(_tid(theory), Nx, Ny, h, _p(p), _p(re), _p(im), _p(out))
    return complex(out[0], out[1])


def gradient(theory, phi, h, params, mode=GRAD_EL) -> np.ndarray:
    """Gradient on interior sites (raw, not projected); zero on the halo.

    mode GRAD_EXACT: h^-2 dE_h/dphi.  mode GRAD_EL: Euler-Lagrange form with eq. (1)-(2).
    """
    phi, p = _arr(phi), _arr(params)
    Nx, Ny = _dims(phi)
    G = np.zeros_like(phi)
    lib().or_gradient(_tid(theory), int(mode), Nx, Ny, h, _p(p), _p(phi), _p(G))
    return G


def acceleration(theory, phi, h, params, mode=GRAD_EL) -> np.ndarray:
    """The flow force a(phi) = -G (chiral magnet: at the normalised point, tangent-projected)."""
    phi, p = _arr(phi), _arr(params)
    Nx, Ny = _dims(phi)
    a = np.zeros_like(phi)
    lib().or_acceleration(_tid(theory), int(mode), Nx, Ny, h, _p(p), _p(phi), _p(a))
    return a


def flow(theory, phi, v, h, params, n_steps, E_cur=None, courant=COURANT, mode=GRAD_EL, scheme="rk4"):
    """n_steps of the flow (arrested Newton flow by RK4 or velocity Verlet, or gradient
    flow: scheme "rk4", "vv", "gf"). Returns (phi, v, E, n_arrests) (new arrays)."""
    phi, v, p = _arr(phi).copy(), _arr(v).copy(), _arr(params)
    Nx, Ny = _dims(phi)
    if E_cur is None:
        E_cur = energy(theory, phi, h, params)
    E = ctypes.c_double(E_cur)
    na = ctypes.c_long(0)
    lib().or_flow_scheme(_tid(theory), int(mode), SCHEMES[scheme], Nx, Ny, h, _p(p), courant, _p(phi), _p(v),
                         ctypes.byref(E), int(n_steps), ctypes.byref(na))
    return phi, v, E.value, na.value


def minimise(theory, phi, h, params, grad_tol=1e-6, rel_e_tol=0.0, window=0, max_steps=100000,
             v=None, courant=COURANT, mode=GRAD_EL, scheme="rk4"):
    """The flow (scheme as in flow) to a stop criterion. Returns (phi, v, info dict)."""
    phi, p = _arr(phi).copy(), _arr(params)
    v = np.zeros_like(phi) if v is None else _arr(v).copy()
    Nx, Ny = _dims(phi)
    info = np.zeros(6)
    lib().or_minimise_scheme(_tid(theory), int(mode), SCHEMES[scheme], Nx, Ny, h, _p(p), courant, _p(phi), _p(v),
                             grad_tol, rel_e_tol, int(window), int(max_steps), _p(info))
    return phi, v, {"E": info[0], "gmax": info[1], "steps": int(info[2]), "arrests": int(info[3]),
                    "converged": bool(info[4]), "reason": int(info[5])}


def poisson(rhs, h) -> np.ndarray:
    """psi with Laplace_h psi = rhs on the interior ((Ny, Nx) arrays), eq. (2) Laplacian,
    psi = 0 outside the interior (conjugate gradients to 1e-14)."""
    rhs = _arr(rhs)
    Ny, Nx = rhs.shape
    out = np.zeros_like(rhs)
    lib().or_poisson(Nx, Ny, h, _p(rhs), _p(out))
    return out


def observables(theory, phi, h, params) -> dict:
    phi, p = _arr(phi), _arr(params)
    Nx, Ny = _dims(phi)
    if _tid(theory) == 6:
        out = np.zeros(3)
        lib().or_observables_bec(Nx, Ny, h, _p(p), _p(phi), _p(out))
        return {"E": out[0], "N": out[1], "Lz": out[2]}
    if _tid(theory) == 0:
        out = np.zeros(6)
        lib().or_observables_ah(Nx, Ny, h, _p(p), _p(phi), _p(out))
        return {"E": out[0], "flux": out[1], "N_rho": out[2], "N_wind": out[3], "R1": out[4], "R2": out[5]}
    out = np.zeros(3)
    lib().or_observables_unit(_tid(theory), Nx, Ny, h, _p(p), _p(phi), _p(out))
    return {"E": out[0], "Q_fd": out[1], "Q_bl": out[2]}


__all__ = ["build", "lib", "energy", "energy_density", "energy_complex", "gradient", "acceleration",
           "flow", "minimise", "observables", "deriv_at", "poisson", "THEORIES", "COURANT", "GRAD_EXACT", "GRAD_EL", "SCHEMES"]
