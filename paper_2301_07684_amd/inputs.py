"""Seeded synthetic particle/field ensembles for the QED step (numpy only).

This module holds no part of the method's arithmetic: it only draws momenta, fields and ids
with the shapes and distributions of the workloads (the paper uses no public data set; all
inputs are synthetic).  Values are counter-based -- particle i of a workload is a pure function
of (workload seed, stream, i) via the splitmix64 finaliser -- so any subsample can be generated
without the full ensemble, and the test oracle and the GPU path see identical inputs.

Workloads (normalised units: lambda = 0.8 um laser wavelength sets omega_r = 2 pi c / lambda):
  plain_compton     65,536 electrons; gamma log-uniform [1e2, 1e5]; isotropic directions; E = 0;
                    B perpendicular to p with random azimuth and |B| set so that the target chi
                    is log-uniform [1e-3, 1e2]; dt = 0.01 fs
  plane_wave        electrons and photons counter-propagating (along -x) through a linearly
                    polarised plane wave along +x: E = a cos(phi) y, B = a cos(phi) z with
                    a ~ U[10, 500], phi ~ U[0, 2 pi); gamma log-uniform [1e2, 1e5]
  plane_wave_skewed the same geometry with a |cos phi| set so that chi is log-uniform [1e-4, 1e3]
  tiles             uneven tiles (sizes log-uniform [1e3, 4e6]) of electrons, positrons and
                    photons in the plain_compton geometry (chi log-uniform [1e-3, 1e2])
"""
from __future__ import annotations

import math

import numpy as np

LASER_WAVELENGTH = 0.8e-6                      # m
C_LIGHT = 299792458.0                          # m/s
LAMBDA_C = 3.8615926796e-13                    # m, CODATA 2018 reduced Compton wavelength
OMEGA_R = 2.0 * math.pi * C_LIGHT / LASER_WAVELENGTH
LAMBDA_R = C_LIGHT / OMEGA_R
LC_OVER_LR = LAMBDA_C / LAMBDA_R               # converts a target chi into a field strength
DT_SECONDS = 1e-17                             # 0.01 fs
DT = DT_SECONDS * OMEGA_R                      # in units of 1/omega_r

ELECTRON, POSITRON, PHOTON = 0, 1, 2

SEED_PLAIN, SEED_WAVE, SEED_SKEW, SEED_TILES, SEED_SERVE = 101, 102, 103, 104, 105

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix(z: np.ndarray) -> np.ndarray:
    """splitmix64 finaliser (Steele, Lea, Flood 2014) on uint64 arrays."""
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def uniforms(seed: int, stream: int, idx: np.ndarray) -> np.ndarray:
    """Uniform doubles in (0, 1) for particle indices idx of a (seed, stream) pair."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = _mix(np.uint64((seed * 1000003 + stream * 7919) & 0xFFFFFFFFFFFFFFFF))
        z = _mix(key + idx * np.uint64(0x9E3779B97F4A7C15))
    return ((z >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53


def ids(seed: int, idx: np.ndarray) -> np.ndarray:
    """Distinct 63-bit particle ids (int64 bit patterns) for indices idx."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return ((np.uint64(seed) << np.uint64(40)) + idx).astype(np.int64)


def _loguniform(u, lo, hi):
    return 10.0 ** (np.log10(lo) + (np.log10(hi) - np.log10(lo)) * u)


def _isotropic(seed, stream, idx):
    ct = 2.0 * uniforms(seed, stream, idx) - 1.0
    ph = 2.0 * math.pi * uniforms(seed, stream + 1, idx)
    st = np.sqrt(np.maximum(0.0, 1.0 - ct * ct))
    return np.stack([st * np.cos(ph), st * np.sin(ph), ct])


def _perp_unit(d, seed, stream, idx):
    """A unit vector perpendicular to d (3, n) with uniform azimuth."""
    a = np.where(np.abs(d[0]) < 0.9, 1.0, 0.0)
    helper = np.stack([a, 1.0 - a, np.zeros_like(a)])
    e1 = np.cross(d.T, helper.T).T
    e1 /= np.linalg.norm(e1, axis=0)
    e2 = np.cross(d.T, e1.T).T
    ph = 2.0 * math.pi * uniforms(seed, stream, idx)
    return np.cos(ph) * e1 + np.sin(ph) * e2


def plain_compton(n: int = 65536, idx=None, seed: int = SEED_PLAIN, species: int = ELECTRON,
                  chi_range=(1e-3, 1e2), gamma_range=(1e2, 1e5)):
    """Isotropic leptons (or photons) in a static magnetic field perpendicular to p."""
    idx = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    gamma = _loguniform(uniforms(seed, 0, idx), *gamma_range)
    d = _isotropic(seed, 1, idx)
    pm = gamma if species == PHOTON else np.sqrt((gamma - 1.0) * (gamma + 1.0))
    p = d * pm
    chi_t = _loguniform(uniforms(seed, 3, idx), *chi_range)
    b = _perp_unit(d, seed, 4, idx) * (chi_t / (pm * LC_OVER_LR))
    return dict(species=species, p=p, E=np.zeros_like(p), B=b, uid=ids(seed, idx),
                chi_target=chi_t, gamma=gamma)


def plane_wave(n: int, idx=None, seed: int = SEED_WAVE, species: int = ELECTRON,
               chi_range=None, a_range=(10.0, 500.0), gamma_range=(1e2, 1e5)):
    """Particles along -x in the plane wave E = a cos(phi) y, B = a cos(phi) z.

    With chi_range, a |cos phi| is set from a log-uniform target chi instead of drawn."""
    idx = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    stream0 = 10 * (species + 1)
    gamma = _loguniform(uniforms(seed, stream0, idx), *gamma_range)
    pm = gamma if species == PHOTON else np.sqrt((gamma - 1.0) * (gamma + 1.0))
    if chi_range is None:
        a = a_range[0] + (a_range[1] - a_range[0]) * uniforms(seed, stream0 + 1, idx)
        phase = 2.0 * math.pi * uniforms(seed, stream0 + 2, idx)
        amp = a * np.cos(phase)
        chi_t = None
    else:
        chi_t = _loguniform(uniforms(seed, stream0 + 3, idx), *chi_range)
        sign = np.where(uniforms(seed, stream0 + 4, idx) < 0.5, -1.0, 1.0)
        a = sign * chi_t / ((gamma + pm) * LC_OVER_LR)
        phase = np.zeros_like(a)
        amp = a
    z = np.zeros_like(gamma)
    p = np.stack([-pm, z, z])
    E = np.stack([z, amp, z])
    B = np.stack([z, z, amp.copy()])
    # wave_a, wave_phase: the same fields as a plane wave along +x polarised along y,
    # E_y = B_z = wave_a cos(wave_phase)
    return dict(species=species, p=p, E=E, B=B, uid=ids(seed + species, idx), chi_target=chi_t,
                gamma=gamma, wave_a=a, wave_phase=phase)


SEED_GENERAL = 106


def general_fields(n: int, idx=None, seed: int = SEED_GENERAL, species: int = ELECTRON,
                   field_range=(1.0, 1e3), gamma_range=(1e2, 1e5)):
    """Isotropic particles in fields of arbitrary geometry: E and B in independent isotropic
    directions with log-uniform magnitudes (units of m c omega_r / e), for steps that push the
    momentum through the fields before the QED step."""
    idx = np.arange(n, dtype=np.uint64) if idx is None else np.asarray(idx, dtype=np.uint64)
    s0 = 50 + 10 * species
    gamma = _loguniform(uniforms(seed, s0, idx), *gamma_range)
    pm = gamma if species == PHOTON else np.sqrt((gamma - 1.0) * (gamma + 1.0))
    p = _isotropic(seed, s0 + 1, idx) * pm
    E = _isotropic(seed, s0 + 3, idx) * _loguniform(uniforms(seed, s0 + 5, idx), *field_range)
    B = _isotropic(seed, s0 + 6, idx) * _loguniform(uniforms(seed, s0 + 8, idx), *field_range)
    return dict(species=species, p=p, E=E, B=B, uid=ids(seed + species, idx), gamma=gamma)


def tile_sizes(ntiles: int = 64, seed: int = SEED_TILES, lo: float = 1e3, hi: float = 4e6):
    u = uniforms(seed, 90, np.arange(ntiles))
    sizes = np.floor(_loguniform(u, lo, hi)).astype(np.int64)
    order = np.argsort(uniforms(seed, 91, np.arange(ntiles)))
    species = np.array([ELECTRON, POSITRON, PHOTON])[np.arange(ntiles) % 3][order]
    return sizes, species


def tiles(ntiles: int = 64, seed: int = SEED_TILES, scale: float = 1.0):
    """Uneven tiles of mixed species in the plain_compton geometry (sizes scaled by `scale`)."""
    sizes, species = tile_sizes(ntiles, seed)
    out = []
    for k, (n, sp) in enumerate(zip(sizes, species)):
        n = max(1, int(n * scale))
        out.append(plain_compton(n, seed=seed * 1000 + k, species=int(sp)))
    return out


# ------------------------------------------------------------------------------------------------
# The same counter-based draws on a torch device (for ensembles created on the GPU at run time,
# e.g. by the serving harness).  uniforms_t reproduces uniforms() bit for bit; the workload
# formulas below use torch's float64 functions, so they agree with the numpy versions to a few
# ulp rather than exactly.
# ------------------------------------------------------------------------------------------------
def _s64(v: int) -> int:
    """A uint64 constant as the int64 with the same bits."""
    v &= 0xFFFFFFFFFFFFFFFF
    return v - (1 << 64) if v >= (1 << 63) else v


_C1, _C2, _GOLD = _s64(0xBF58476D1CE4E5B9), _s64(0x94D049BB133111EB), _s64(0x9E3779B97F4A7C15)


def _srl(z, k: int):
    """Logical right shift of int64 bit patterns."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def _mix_t(z):
    z = (z ^ _srl(z, 30)) * _C1
    z = (z ^ _srl(z, 27)) * _C2
    return z ^ _srl(z, 31)


def uniforms_t(seed: int, stream: int, idx):
    """uniforms() for an int64 torch tensor of indices (on any device)."""
    import torch

    key = int(_mix(np.uint64((seed * 1000003 + stream * 7919) & 0xFFFFFFFFFFFFFFFF)))
    z = _mix_t(idx * _GOLD + _s64(key))
    return (_srl(z, 11).to(torch.float64) + 0.5) * 2.0 ** -53


def ids_t(seed: int, idx):
    return idx + (seed << 40)


def plane_wave_t(n: int, device, seed: int = SEED_WAVE, species: int = ELECTRON,
                 a_range=(10.0, 500.0), gamma_range=(1e2, 1e5)):
    """plane_wave() generated on `device`: dict of (3, n) float64 tensors p, E, B, int64 uid, and
    the field amplitude a and phase phi of each particle (E_y = B_z = a cos phi)."""
    import torch

    idx = torch.arange(n, dtype=torch.int64, device=device)
    s0 = 10 * (species + 1)
    lo, hi = math.log10(gamma_range[0]), math.log10(gamma_range[1])
    gamma = torch.pow(10.0, lo + (hi - lo) * uniforms_t(seed, s0, idx))
    pm = gamma if species == PHOTON else torch.sqrt((gamma - 1.0) * (gamma + 1.0))
    a = a_range[0] + (a_range[1] - a_range[0]) * uniforms_t(seed, s0 + 1, idx)
    phi = 2.0 * math.pi * uniforms_t(seed, s0 + 2, idx)
    amp = a * torch.cos(phi)
    z = torch.zeros_like(gamma)
    return dict(species=species, p=torch.stack([-pm, z, z]), E=torch.stack([z, amp, z]),
                B=torch.stack([z, z, amp]), uid=ids_t(seed + species, idx), a=a, phi=phi)


# ---- constant-field validation set-up (paper Sec. 4.3: 10 GeV electrons at chi = 1 in a constant,
# uniform magnetic field, 1.3 fs) ------------------------------------------------------------------
ELECTRON_REST_MEV = 0.51099895000
GAMMA_10GEV = 1.0e4 / ELECTRON_REST_MEV
T_SIM_FS = 1.3
SEED_SYNC = 107


def synchrotron_t(n: int, device, seed: int = SEED_SYNC, gamma: float = GAMMA_10GEV,
                  chi: float = 1.0):
    """n electrons of energy gamma moving along +x in the uniform field B = b z with b set so
    that chi = lambda_C |p| b / lambda_r.  Returns torch tensors: p (3, n) float64 and uid (n,)
    int64 on `device`, and the one-element field arrays E (3 x zeros) and B (0, 0, b) for
    tiles with uniform fields."""
    import torch

    pm = math.sqrt((gamma - 1.0) * (gamma + 1.0))
    b = chi / (pm * LC_OVER_LR)
    f = lambda v: torch.full((1,), v, dtype=torch.float64, device=device)
    p = torch.zeros((3, n), dtype=torch.float64, device=device)
    p[0].fill_(pm)
    uid = ids_t(seed, torch.arange(n, dtype=torch.int64, device=device))
    return dict(p=p, uid=uid, E=[f(0.0), f(0.0), f(0.0)], B=[f(0.0), f(0.0), f(b)], b=b, pm=pm)
