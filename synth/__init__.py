"""Seeded synthetic inputs for the constraint solve.

This module only draws random numbers and fixes workload parameters: the
wavevectors, phases and amplitudes of the scalar-field Fourier modes, grid
sizes and box geometry.  It evaluates no field and computes no density,
residual or operator: both the CPU oracle and the GPU library turn these
tables into sources (rho, S_i) on their own.

Workloads (scalar-field matter, the paper's periodic-cosmology and
black-hole scenarios, Key features):

* ``hamiltonian_32``  periodic cube L=1, 32^3, 4 levels, 3 modes of
  amplitude 0.01, Pi = 0, plain FP64, momentum trivial.
* ``coupled_128``     periodic cube L=1, 128^3, 6 levels, phi: 8 modes of
  amplitude 0.05; Pi: 8 modes of amplitude 0.02 (own stream).
* ``puncture_shell``  box [-32,32]^3, M=1 puncture at the centre, scalar
  shell phi = 0.1 exp(-(r-10)^2/4) Y_11, Pi = 0, Robin outer boundary; the
  shell's density is taken as conformally rescaled free data.
* ``scan_96``         96 periodic instances, N uniform on {32,48,64,96},
  phi amplitude uniform on [0.01, 0.1], Pi amplitude 0.02.

Mode tables are float64 arrays of shape (count, 5): kx, ky, kz (integers
stored as float), amplitude, phase.  A field is meant as
sum_m amp_m * cos(2 pi k_m . x / L + phase_m).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

BC_PERIODIC = 0
BC_ROBIN = 1
PREC_FP64 = 0
PREC_FP32_IR = 1


def wavevectors(kmax: int = 3) -> np.ndarray:
    """All integer vectors k with 0 < |k|^2 <= kmax^2, in a fixed order (122 for kmax=3)."""
    out = []
    r = range(-kmax, kmax + 1)
    for a in r:
        for b in r:
            for c in r:
                q = a * a + b * b + c * c
                if 0 < q <= kmax * kmax:
                    out.append((a, b, c))
    return np.asarray(out, dtype=np.int64)


def fourier_modes(rng: np.random.Generator, count: int, amplitude: float) -> np.ndarray:
    """Draw ``count`` distinct wavevectors uniformly from ``wavevectors()``, with
    uniform phases on [0, 2 pi) and a common amplitude."""
    ks = wavevectors()
    pick = rng.choice(len(ks), size=count, replace=False)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=count)
    tab = np.zeros((count, 5), dtype=np.float64)
    tab[:, 0:3] = ks[pick]
    tab[:, 3] = amplitude
    tab[:, 4] = phases
    return tab


@dataclasses.dataclass
class Workload:
    """One initial-data instance: geometry, solver options and matter draws."""
    name: str
    n: int
    levels: int
    length: float = 1.0
    origin: tuple = (0.0, 0.0, 0.0)
    bc: int = BC_PERIODIC
    precision: int = PREC_FP64
    solve_momentum: bool = False
    nu_pre: int = 2
    nu_post: int = 2
    # W V-cycle sweeps while its bottom is exact (0: nu_pre / nu_post)
    nu_pre_W: int = 0
    nu_post_W: int = 0
    # corrections prolonged by the 4-point cubic instead of trilinearly
    cubic_prolong: bool = False
    # both steps of an outer iteration linearised at the state it starts from
    same_state: bool = False
    # steps the CTTK solve's Anderson mixing combines (0 or 1: one step)
    mix_depth: int = 0
    scalar_mass: float = 1.0
    phi_modes: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 5)))
    pi_modes: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 5)))
    # puncture + shell scenario
    puncture_mass: float = 0.0
    puncture_pos: tuple = (0.0, 0.0, 0.0)
    shell: Optional[dict] = None
    # sources given as conformally rescaled rho_bar = psi^8 rho, S_bar = psi^6 S
    conformal_matter: bool = False
    # Bowen-York punctures: rows (m, C[3], P[3], S[3]); None when not used
    punctures: Optional[np.ndarray] = None
    seed: Optional[int] = None
    tol: float = 1e-10

    @property
    def h(self) -> float:
        return self.length / self.n


def coarsest_levels(n: int) -> int:
    """Number of levels when halving while n is even and n/2 >= 3."""
    lv = 1
    while n % 2 == 0 and n // 2 >= 3:
        n //= 2
        lv += 1
    return lv


def hamiltonian_32(seed: int = 0) -> Workload:
    rng = np.random.default_rng(seed)
    return Workload(name="hamiltonian_32", n=32, levels=4, seed=seed,
                    phi_modes=fourier_modes(rng, 3, 0.01),
                    precision=PREC_FP64, solve_momentum=False)


def coupled(n: int = 128, seed: int = 0, phi_amp: float = 0.05,
            precision: int = PREC_FP32_IR, levels: Optional[int] = None) -> Workload:
    rng_phi = np.random.default_rng(seed)
    rng_pi = np.random.default_rng([seed, 1])
    # Corrections prolonged by the 4-point cubic, both steps of an outer iteration from its
    # starting state (one finest residual per iteration, the two V-cycles side by side), psi
    # V(1,3) and W V(1,2) while its bottom is exact: the fastest to rms 1e-10 at 128^3 measured
    # (mixed, FMG start / zero start: psi V(1,3) W V(1,2) 3.52 / 3.98 ms; W V(2,1) 3.60 / 4.06;
    # psi V(2,2) W V(2,1) 3.72-3.78 / 4.11-4.19; psi V(1,2) W V(1,1) 3.76-3.97 / 3.87-3.92 with
    # 10 iterations; psi V(1,4) 3.94 / 4.42; the two steps in sequence with V(2,2) 4.78 / 4.85).
    # FP64 (the W cycle with the psi sweeps): V(1,3) 10.27 ms / 10 iterations, V(2,2) 10.50,
    # V(1,2) 10.21 / 12, V(2,1) 10.49 / 12.  CTTK on this workload mixes the last 3 W steps
    # (128^3: 20.8 ms / 39 iterations; one step 23.4 / 51, 5 steps 21.1 / 34, 6 steps 23.4 / 35:
    # each stored step costs two more passes over 3 n^3 doubles per iteration).
    return Workload(name=f"coupled_{n}", n=n,
                    levels=levels if levels is not None else coarsest_levels(n),
                    seed=seed, phi_modes=fourier_modes(rng_phi, 8, phi_amp),
                    pi_modes=fourier_modes(rng_pi, 8, 0.02),
                    precision=precision, solve_momentum=True, nu_pre=1, nu_post=3, nu_pre_W=1, nu_post_W=2,
                    cubic_prolong=True, same_state=True, mix_depth=3)


def coupled_128(seed: int = 0, precision: int = PREC_FP32_IR) -> Workload:
    return coupled(128, seed, 0.05, precision)


def puncture_shell(n: int = 256, precision: int = PREC_FP32_IR,
                   levels: int = 6) -> Workload:
    # cubic prolongation of corrections: 5 outer iterations at 256^3 (19.1 ms) against 8 (31.3)
    return Workload(name=f"puncture_shell_{n}", n=n, levels=levels, length=64.0,
                    origin=(-32.0, -32.0, -32.0), bc=BC_ROBIN, precision=precision,
                    solve_momentum=False, puncture_mass=1.0,
                    puncture_pos=(0.0, 0.0, 0.0), conformal_matter=True,
                    shell=dict(amplitude=0.1, r0=10.0, width2=4.0), cubic_prolong=True)


def bowen_york_binary(n: int = 256, precision: int = PREC_FP32_IR, levels: int = 6) -> Workload:
    """Two unequal boosted and spinning punctures in vacuum on the box [-32, 32]^3
    (the 64 M box of the isolated black-hole workload), Robin boundaries about
    the centre, K = 0.  The punctures sit on cell vertices of every grid with
    h dividing 1 (n = 64, 128, 256)."""
    table = np.array([
        [0.5, 3.0, 0.0, 0.0, 0.0, 0.1, 0.0, 0.0, 0.0, 0.2],
        [0.5, -3.0, 0.0, 0.0, 0.0, -0.1, 0.0, 0.05, 0.0, -0.1],
    ])
    # cubic prolongation of corrections: 5 outer iterations at 256^3 (19.7 ms) against 8 (32.4)
    return Workload(name=f"bowen_york_binary_{n}", n=n, levels=levels, length=64.0,
                    origin=(-32.0, -32.0, -32.0), bc=BC_ROBIN, precision=precision,
                    solve_momentum=False, punctures=table, cubic_prolong=True)


def scan_96(count: int = 96, size_seed: int = 12345,
            sizes=(32, 48, 64, 96)) -> List[Workload]:
    rng = np.random.default_rng(size_seed)
    ns = rng.choice(np.asarray(sizes), size=count)
    amps = rng.uniform(0.01, 0.1, size=count)
    out = []
    for i in range(count):
        w = coupled(int(ns[i]), seed=i, phi_amp=float(amps[i]), precision=PREC_FP32_IR)
        w.name = f"scan_{i}"
        out.append(w)
    return out


def random_smooth_field(seed: int, n: int, count: int = 4, amplitude: float = 0.1) -> np.ndarray:
    """A mode table for a smooth periodic test field (initial guesses, forcing)."""
    return fourier_modes(np.random.default_rng([seed, 7]), count, amplitude)


def uniform_random(seed: int, shape, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Plain seeded uniform noise (float64), for operator-level parity inputs."""
    return np.random.default_rng([seed, 11]).uniform(lo, hi, size=shape)


def nn_init(shapes, seed: int, bias_scale: float = 0.0) -> np.ndarray:
    """Seeded initial parameters of a stack of 3x3x3 convolutions, laid out per layer
    as W[co][ci][3][3][3] then b[co] (float32): W ~ N(0, 2 / (27 ci)) (He
    initialisation), b ~ U(-bias_scale, bias_scale)."""
    rng = np.random.default_rng([seed, 23])
    parts = []
    for ci, co in shapes:
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (27.0 * ci)), size=27 * ci * co))
        parts.append(rng.uniform(-bias_scale, bias_scale, size=co) if bias_scale > 0 else np.zeros(co))
    return np.concatenate(parts).astype(np.float32)
