"""Seeded synthetic inputs for the three-layer Rayleigh-Taylor workloads.

This module holds parameters and random draws only -- none of the method's
arithmetic -- so that the product path and the CPU oracle can be fed the same
inputs.  It imports nothing from the rest of the package.

Workloads (lattice sizes and physics of the double-front run of Sec. IV,
Table II, scaled to the measured shapes):

  rt3_128x384        FP64, 100 steps; the small case the oracle finishes
  rt3_4096x12288     FP64, one GPU's production share (~50 M sites)
  rt3_4096x12288_f32 the same lattice with FP32 deviation storage
  rt3_512x1536_adj   FP64 with 32 interface modes differentiated
  rt3_2048x6144_adj  FP32 storage forward + adjoint
  rt3_2400x6144_paper / rt2_2400x6144_paper
                     the double- and single-front runs of Sec. IV (Table II)

Physics common to all: tau = 0.7, temperatures 1.05 / 1.00 / 0.95 (bottom,
middle, top) in equal thirds, tanh half-width 4 sites, 16 Fourier modes per
interface with wavenumbers 1..16, phases U[0, 2 pi), amplitudes U[0, 1] site.
Gravity keeps g * Lz fixed at 1e-4 * 384 (negligible stratification, as in
Sec. IV): g = 1e-4 at Lz = 384.
"""
from dataclasses import dataclass

import numpy as np

NMODES = 16


@dataclass(frozen=True)
class Workload:
    name: str
    lx: int
    lz: int
    steps: int
    precision: str            # "f64" or "f32dev"
    seed: int
    tau: float = 0.7
    t_d: float = 1.05
    t_m: float = 1.00
    t_u: float = 0.95
    width: float = 4.0
    ckpt_every: int = 0       # adjoint workloads: state checkpoint interval (0: as many
                              # steps as the kept moments cover)
    adj_precision: str = "f64"  # adjoint workloads: "f32" = float adjoint buffers
    z_lo: float = None        # interface rest heights (sites); None: Lz/3, 2 Lz/3
    z_hi: float = None
    g_override: float = None  # gravity when not scaled with Lz
    t_m_diag: float = None    # middle temperature of the tent-map diagnostics
                              # (the single-front run's "virtual" T_m)
    wall: str = "dirichlet"   # wall rule: "dirichlet" or "diffuse" (mass-conserving)
    inplace: bool = False     # single population buffer (lbm_step_inplace)
    mom_precision: str = "f64"  # adjoint workloads: "f32" = stored moments in float

    @property
    def g(self) -> float:
        return self.g_override if self.g_override is not None else 1e-4 * 384.0 / self.lz

    @property
    def atwood(self) -> float:
        return (self.t_d - self.t_u) / (self.t_d + self.t_u)

    @property
    def sites(self) -> int:
        return self.lx * self.lz


WORKLOADS = {
    w.name: w for w in (
        Workload("rt3_128x384", 128, 384, 100, "f64", 1405),
        Workload("rt3_4096x12288", 4096, 12288, 1000, "f64", 1405),
        Workload("rt3_4096x12288_f32", 4096, 12288, 20000, "f32dev", 1405),
        Workload("rt3_512x1536_adj", 512, 1536, 2000, "f64", 1253, ckpt_every=100),
        Workload("rt3_4096x12288_diffuse", 4096, 12288, 1000, "f64", 1405, wall="diffuse"),
        Workload("rt3_4096x12288_f32_diffuse", 4096, 12288, 20000, "f32dev", 1405, wall="diffuse"),
        Workload("rt3_512x1536_adj_diffuse", 512, 1536, 2000, "f64", 1253, ckpt_every=100,
                 wall="diffuse"),
        Workload("rt3_4096x12288_inplace", 4096, 12288, 1000, "f64", 1405, inplace=True),
        Workload("rt3_4096x12288_f32_inplace", 4096, 12288, 20000, "f32dev", 1405, inplace=True),
        # the largest lattice the library accepts (2^29 sites): one FP64
        # buffer of 159 GB; two would not fit in one GPU's 288 GB
        Workload("rt3_16384x32768_inplace", 16384, 32768, 1000, "f64", 1405, inplace=True),
        Workload("rt3_2048x6144_adj", 2048, 6144, 5000, "f32dev", 1405, ckpt_every=0,
                 adj_precision="f32", mom_precision="f32"),
        # The runs of Sec. IV, Table II: 2400 x 6144, g = 1.5e-5, T 1.025/1/0.975,
        # a middle layer delta = 500 for the double front; Ra = 1e10 at Pr = 1
        # gives nu = sqrt(dT Lz^3 g / Ra) = 5.46e-3 with Lz in length units.
        Workload("rt3_2400x6144_paper", 2400, 6144, 350000, "f32dev", 1405, tau=0.50546,
                 t_d=1.025, t_m=1.0, t_u=0.975, z_lo=3072 - 250, z_hi=3072 + 250,
                 g_override=1.5e-5),
        Workload("rt2_2400x6144_paper", 2400, 6144, 350000, "f32dev", 1405, tau=0.50546,
                 t_d=1.025, t_m=1.025, t_u=0.975, z_lo=1536, z_hi=3072, g_override=1.5e-5,
                 t_m_diag=1.0),
    )
}


@dataclass
class Modes:
    k: np.ndarray       # int32 [2, NMODES]  (front 0: lower interface, 1: upper)
    phase: np.ndarray   # float64 [2, NMODES]
    amp: np.ndarray     # float64 [2, NMODES]


def draw_modes(seed: int, nmodes: int = NMODES) -> Modes:
    """Wavenumbers 1..nmodes on both fronts; phases then amplitudes drawn with
    numpy PCG64 default_rng(seed), lower front first."""
    rng = np.random.default_rng(seed)
    k = np.tile(np.arange(1, nmodes + 1, dtype=np.int32), (2, 1))
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(2, nmodes))
    amp = rng.uniform(0.0, 1.0, size=(2, nmodes))
    return Modes(k, phase, amp)


def fd_mode_indices(seed: int = 1254, count: int = 8) -> np.ndarray:
    """Flat indices (front * NMODES + j) of the modes checked by finite differences."""
    return np.random.default_rng(seed).choice(2 * NMODES, count, replace=False)


def random_populations(seed: int, lx: int, lz: int, lo: float = 0.5,
                       hi: float = 1.5, q: int = 37) -> np.ndarray:
    """Uniform random float64 field [q, lx, lz] for streaming tests."""
    return np.random.default_rng(seed).uniform(lo, hi, size=(q, lx, lz))


def random_ghost(seed: int, q: int = 37) -> np.ndarray:
    """Uniform random wall table [2, 3, q] for streaming tests."""
    return np.random.default_rng(seed).uniform(2.0, 3.0, size=(2, 3, q))
