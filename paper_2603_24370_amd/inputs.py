"""Seeded synthetic inputs for the soliton flow: lattices, ansatz fields and noise.

This module only builds starting configurations and instance descriptions. It
contains none of the solver's arithmetic (no stencil, no energy, no gradient, no
time step), so both the CPU oracle and the HIP path can consume what it makes.

Layout of every field array: planar, component-major, row-major with x fastest,
shape ``(C, Ny + 4, Nx + 4)`` including the width-2 halo of Sec. 3.1 of the paper.
Interior site (i, j) sits at array index ``[c, j + 2, i + 2]``.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based generator:
draw ``n`` of stream ``key`` is ``mix(key + (n + 1) * GOLDEN)``, with ``mix`` the
SplitMix64 output function. ``key`` itself is ``mix(seed * GOLDEN + stream)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

HALO = 2
GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# Stream identifiers, so that independent draws never share counters.
STREAM_NOISE = 1
STREAM_INSTANCE = 2
STREAM_CENTRES = 3
STREAM_DISC = 4


def _mix(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on uint64 arrays (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GOLDEN + np.uint64(stream)
    return np.uint64(_mix(np.array([s], dtype=np.uint64))[0])


def uniform01(seed: int, stream: int, counters: np.ndarray) -> np.ndarray:
    """Doubles in [0, 1) for the given uint64 counters of one stream."""
    key = stream_key(seed, stream)
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = _mix(key + (c + np.uint64(1)) * GOLDEN)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def coords(n: int, h: float) -> np.ndarray:
    """Cell-centred coordinates of all n + 4 padded sites along one axis."""
    idx = np.arange(-HALO, n + HALO, dtype=np.float64)
    return (idx - (n - 1) / 2.0) * h


def grid(Nx: int, Ny: int, h: float):
    x = coords(Nx, h)
    y = coords(Ny, h)
    X, Y = np.meshgrid(x, y)  # shape (Ny+4, Nx+4), x fastest
    return X, Y


def interior_mask(Nx: int, Ny: int) -> np.ndarray:
    m = np.zeros((Ny + 2 * HALO, Nx + 2 * HALO), dtype=bool)
    m[HALO:HALO + Ny, HALO:HALO + Nx] = True
    return m


def noise(seed: int, C: int, Nx: int, Ny: int, amp: float) -> np.ndarray:
    """U(-amp, amp) per interior site and component, zero on the halo.

    Counter of (c, j, i) is ``(c * Ny + j) * Nx + i`` on the noise stream.
    """
    out = np.zeros((C, Ny + 2 * HALO, Nx + 2 * HALO), dtype=np.float64)
    c = np.arange(C, dtype=np.uint64)[:, None, None]
    j = np.arange(Ny, dtype=np.uint64)[None, :, None]
    i = np.arange(Nx, dtype=np.uint64)[None, None, :]
    ctr = (c * np.uint64(Ny) + j) * np.uint64(Nx) + i
    u = uniform01(seed, STREAM_NOISE, ctr)
    out[:, HALO:HALO + Ny, HALO:HALO + Nx] = amp * (2.0 * u - 1.0)
    return out


# ---------------------------------------------------------------------------
# Abelian-Higgs / Ginzburg-Landau product ansatz (fields psi_1, psi_2, A_1, A_2)
# ---------------------------------------------------------------------------

def ah_vortex_ansatz(Nx: int, Ny: int, h: float, centres, windings=None,
                     halo: str = "vacuum") -> np.ndarray:
    """psi = prod_k tanh(r_k) exp(i n_k theta_k),  A = sum_k n_k (1-exp(-r_k^2))/r_k^2 (-(y-y_k), x-x_k).

    ``halo='vacuum'`` fills the halo with the pure-gauge vacuum of the same
    winding, psi = exp(i sum n_k theta_k), A = sum n_k grad theta_k; ``'ansatz'``
    keeps the ansatz there too. Returns float64 of shape (4, Ny+4, Nx+4).
    """
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 2)
    if windings is None:
        windings = np.ones(len(centres), dtype=np.float64)
    windings = np.asarray(windings, dtype=np.float64)
    X, Y = grid(Nx, Ny, h)
    mod = np.ones_like(X)
    phase = np.zeros_like(X)
    A1 = np.zeros_like(X)
    A2 = np.zeros_like(X)
    V1 = np.zeros_like(X)
    V2 = np.zeros_like(X)
    for (xk, yk), nk in zip(centres, windings):
        dx = X - xk
        dy = Y - yk
        r2 = dx * dx + dy * dy
        r = np.sqrt(r2)
        mod = mod * np.tanh(r)
        phase = phase + nk * np.arctan2(dy, dx)
        safe = np.where(r2 > 1e-300, r2, 1.0)
        prof = np.where(r2 > 1e-300, -np.expm1(-r2) / safe, 1.0)
        A1 += nk * prof * (-dy)
        A2 += nk * prof * dx
        V1 += nk * (-dy) / safe
        V2 += nk * dx / safe
    out = np.stack([mod * np.cos(phase), mod * np.sin(phase), A1, A2])
    if halo == "vacuum":
        m = ~interior_mask(Nx, Ny)
        out[0][m] = np.cos(phase)[m]
        out[1][m] = np.sin(phase)[m]
        out[2][m] = V1[m]
        out[3][m] = V2[m]
    elif halo != "ansatz":
        raise ValueError(f"unknown halo kind {halo!r}")
    return out


# ---------------------------------------------------------------------------
# Chiral magnet: Belavin-Polyakov skyrmion (unit field n_1, n_2, n_3)
# ---------------------------------------------------------------------------

def cm_skyrmion_ansatz(Nx: int, Ny: int, h: float, R: float = 2.0,
                       gamma: float = -math.pi / 2, centre=(0.0, 0.0),
                       profile: str = "bp", vorticity: int = 1) -> np.ndarray:
    """n = (sin T cos(m th+gamma), sin T sin(m th+gamma), cos T), halo n = e_3,
    m the vorticity (-1: antiskyrmion).

    ``profile='bp'``: T = 2 arctan(R / r) (Belavin-Polyakov).
    ``profile='gauss'``: T = pi exp(-(r/R)^2), a fast-decaying test texture.
    """
    X, Y = grid(Nx, Ny, h)
    dx = X - centre[0]
    dy = Y - centre[1]
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx)
    if profile == "bp":
        T = 2.0 * np.arctan2(R, r)
    elif profile == "gauss":
        T = math.pi * np.exp(-(r / R) ** 2)
    else:
        raise ValueError(profile)
    az = vorticity * th + gamma
    out = np.stack([np.sin(T) * np.cos(az), np.sin(T) * np.sin(az), np.cos(T)])
    m = ~interior_mask(Nx, Ny)
    out[0][m] = 0.0
    out[1][m] = 0.0
    out[2][m] = 1.0
    return out


# ---------------------------------------------------------------------------
# Rotating trapped BEC: Gaussian cloud with optional vortices (psi = u + i w)
# ---------------------------------------------------------------------------

def bec_ansatz(Nx: int, Ny: int, h: float, R: float = 1.0, centres=(), windings=None,
               xi: float = 1.0) -> np.ndarray:
    """psi = exp(-r^2 / (2 R^2)) / (sqrt(pi) R) * prod_k tanh(r_k / xi) exp(i n_k theta_k)
    on the interior, psi = 0 on the halo. Returns float64 of shape (2, Ny+4, Nx+4)."""
    centres = np.asarray(centres, dtype=np.float64).reshape(-1, 2)
    if windings is None:
        windings = np.ones(len(centres), dtype=np.float64)
    X, Y = grid(Nx, Ny, h)
    amp = np.exp(-(X * X + Y * Y) / (2.0 * R * R)) / (math.sqrt(math.pi) * R)
    phase = np.zeros_like(X)
    for (xk, yk), nk in zip(centres, np.asarray(windings, dtype=np.float64)):
        dx, dy = X - xk, Y - yk
        amp = amp * np.tanh(np.hypot(dx, dy) / xi)
        phase = phase + nk * np.arctan2(dy, dx)
    out = np.stack([amp * np.cos(phase), amp * np.sin(phase)])
    out[:, ~interior_mask(Nx, Ny)] = 0.0
    return out


def renormalise_interior(n: np.ndarray) -> np.ndarray:
    """Rescale each interior 3-vector to unit length (input preparation only)."""
    Ny, Nx = n.shape[1] - 2 * HALO, n.shape[2] - 2 * HALO
    out = n.copy()
    sl = (slice(None), slice(HALO, HALO + Ny), slice(HALO, HALO + Nx))
    v = out[sl]
    out[sl] = v / np.sqrt((v * v).sum(axis=0, keepdims=True))
    return out


# ---------------------------------------------------------------------------
# Vortex positions
# ---------------------------------------------------------------------------

def uniform_centres(seed: int, n: int, half_width: float, stream: int = STREAM_CENTRES):
    u = uniform01(seed, stream, np.arange(2 * n, dtype=np.uint64)).reshape(n, 2)
    return (2.0 * u - 1.0) * half_width


def poisson_disc(seed: int, n: int, min_sep: float, half_width: float, max_tries: int = 1_000_000):
    """Dart throwing: accept a uniform candidate if it keeps ``min_sep`` from all accepted."""
    pts = np.zeros((0, 2))
    ctr = 0
    batch = 4096
    while len(pts) < n:
        if ctr >= 2 * max_tries:
            raise RuntimeError("poisson_disc: could not place all points")
        u = uniform01(seed, STREAM_DISC, np.arange(ctr, ctr + 2 * batch, dtype=np.uint64)).reshape(batch, 2)
        ctr += 2 * batch
        for p in (2.0 * u - 1.0) * half_width:
            if len(pts) == 0 or np.min(np.hypot(*(pts - p).T)) >= min_sep:
                pts = np.vstack([pts, p])
                if len(pts) == n:
                    break
    return pts


# ---------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------

def gl_lambda_from_kappa(kappa: float) -> float:
    """Textbook GL relation in units u = e = 1: lambda/8 = kappa^2/4, so lambda = 2 kappa^2."""
    return 2.0 * kappa * kappa


@dataclass
class Instance:
    theory: str
    Nx: int
    Ny: int
    h: float
    params: list
    centres: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))
    seed: int = 0
    noise_amp: float = 1e-3
    kappa: float = float("nan")

    def field(self) -> np.ndarray:
        if self.theory == "abelian_higgs":
            f = ah_vortex_ansatz(self.Nx, self.Ny, self.h, self.centres)
            return f + noise(self.seed, 4, self.Nx, self.Ny, self.noise_amp)
        f = cm_skyrmion_ansatz(self.Nx, self.Ny, self.h, R=2.0, gamma=-math.pi / 2)
        return renormalise_interior(f + noise(self.seed, 3, self.Nx, self.Ny, self.noise_amp))


def ah_single_vortex(N: int = 128, h: float = 0.1, seed: int = 1) -> Instance:
    """Critical AH (lambda = 1), one vortex at the origin, U(+-1e-3) noise."""
    return Instance("abelian_higgs", N, N, h, [1.0], np.zeros((1, 2)), seed)


def cm_single_skyrmion(N: int = 512, h: float = 0.05, seed: int = 2) -> Instance:
    """J = D = 1, K = 0.1, B = 0.6; Belavin-Polyakov R = 2, gamma = -pi/2."""
    return Instance("chiral_magnet", N, N, h, [1.0, 1.0, 0.1, 0.6], np.zeros((0, 2)), seed)


def gl_batch_instance(b: int, base_seed: int = 3000, h: float = 0.2) -> Instance:
    """One of the batched GL instances: side in {64..384 step 32}, kappa ~ U[0.5, 2], N ~ U{1..8}."""
    seed = base_seed + b
    u = uniform01(seed, STREAM_INSTANCE, np.arange(3, dtype=np.uint64))
    side = 64 + 32 * min(int(u[0] * 11), 10)
    kappa = 0.5 + 1.5 * u[1]
    nv = 1 + min(int(u[2] * 8), 7)
    half = 0.5 * 0.6 * side * h
    centres = uniform_centres(seed, nv, half)
    return Instance("abelian_higgs", side, side, h, [gl_lambda_from_kappa(kappa)], centres, seed,
                    kappa=kappa)


def gl_large_instance(N: int = 4096, h: float = 0.2, kappa: float = 1.5, n_vortices: int = 256,
                      seed: int = 4) -> Instance:
    half = 0.5 * 0.6 * N * h
    centres = poisson_disc(seed, n_vortices, 3.0, half)
    return Instance("abelian_higgs", N, N, h, [gl_lambda_from_kappa(kappa)], centres, seed,
                    kappa=kappa)


def blob_map(centres, N: int, h: float, sigma: float = 1.0) -> np.ndarray:
    """Sum of unit Gaussians (width sigma) at the vortex centres on the interior N x N grid."""
    x = coords(N, h)[HALO:HALO + N]
    X, Y = np.meshgrid(x, x)
    out = np.zeros_like(X)
    for xk, yk in np.asarray(centres).reshape(-1, 2):
        out += np.exp(-((X - xk) ** 2 + (Y - yk) ** 2) / (2 * sigma * sigma))
    return out
