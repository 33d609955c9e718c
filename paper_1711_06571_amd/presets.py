"""Named workloads: detector geometry, generator settings and build cuts.

The barrel follows the paper's initial scenario (section 3): concentric
cylinders, uniform longitudinal field, Gaussian-smeared hits, a particle gun
flat in pT between 0.5 and 10 GeV.  The workloads:

* ``fit_small``   -- fit, 1 event x 1 000 tracks, 10 layers at r = 4..40 cm;
* ``fit_scale``   -- fit, 200 events x 20 000 tracks, 17 layers to r = 68 cm;
* ``build``       -- combinatorial build, 20 000 tracks + 20 % noise per layer,
  63 phi x 16 z bins, up to 6 candidates per seed, chi2 < 30, one hole;
* ``batch``       -- 64 events, tracks per event log-uniform in [500, 50 000],
  noise fraction U[0.05, 0.30] per (event, layer);
* ``learned``     -- build workload with the learned search window.

Every physical constant is rounded to FP32 before use so that the simulation
(FP64), the oracle (FP64) and the GPU library (FP32 geometry block) see the
same numbers.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 1711065710


def f32(v: float) -> float:
    return float(np.float32(v))


@dataclass
class Geometry:
    n_layers: int = 10
    r: list = field(default_factory=lambda: [4.0 * (i + 1) for i in range(10)])
    z_half: float = 100.0
    bz: float = f32(3.8)
    x_over_x0: float = f32(0.02)
    mass: float = f32(0.13957)
    # transverse width of the luminous region about the z axis (the
    # generator's vertex spread), used by the seed convention
    beam_sigma: float = f32(0.01)

    def __post_init__(self):
        self.r = [f32(v) for v in self.r]
        self.z_half = f32(self.z_half)
        self.bz = f32(self.bz)
        self.x_over_x0 = f32(self.x_over_x0)
        self.mass = f32(self.mass)
        self.beam_sigma = f32(self.beam_sigma)

    def replace(self, **kw) -> "Geometry":
        return dataclasses.replace(self, **kw)


def barrel(n_layers: int, **kw) -> Geometry:
    return Geometry(n_layers=n_layers, r=[4.0 * (i + 1) for i in range(n_layers)], **kw)


@dataclass
class GenSettings:
    sig_rphi: float = f32(0.01)
    sig_z: float = f32(0.1)
    pt_min: float = 0.5
    pt_max: float = 10.0
    eta_max: float = 1.0
    vtx_sxy: float = 0.01
    vtx_sz: float = 5.0
    noise_lo: float = 0.0
    noise_hi: float = 0.0
    smear: bool = True
    seed: int = SEED_BASE + 1


@dataclass
class BuildCuts:
    chi2_cut: float = 30.0
    max_holes: int = 1
    cand_cap: int = 6
    nsigma: float = 3.0
    win_sig_rphi: float = f32(0.01)
    win_sig_z: float = f32(0.1)
    first_layer: int = 3
    n_phi_bins: int = 63
    n_z_bins: int = 16


@dataclass
class Workload:
    name: str
    geometry: Geometry
    gen: GenSettings
    n_events: int
    n_tracks: int
    cuts: BuildCuts = field(default_factory=BuildCuts)
    tracks_lo: int = 0
    tracks_hi: int = 0


def fit_small() -> Workload:
    return Workload("fit_small: 1 event x 1000 tracks, 10 layers r=4..40 cm, Bz=3.8 T",
                    barrel(10), GenSettings(seed=SEED_BASE + 1), 1, 1000)


def fit_scale() -> Workload:
    return Workload("fit_scale: 200 events x 20000 tracks, 17 layers r=4..68 cm, Bz=3.8 T",
                    barrel(17), GenSettings(seed=SEED_BASE + 2), 200, 20000)


def build() -> Workload:
    return Workload("build: 1 event x 20000 tracks + 20% noise/layer, 17 layers, 63x16 bins, cap 6, chi2<30, 1 hole",
                    barrel(17), GenSettings(seed=SEED_BASE + 3, noise_lo=0.2, noise_hi=0.2), 1, 20000)


def batch() -> Workload:
    return Workload("batch: 64 events, tracks log-uniform [500,50000], noise U[0.05,0.30]/layer/event, 17 layers",
                    barrel(17), GenSettings(seed=SEED_BASE + 4, noise_lo=0.05, noise_hi=0.30), 64, 0,
                    tracks_lo=500, tracks_hi=50000)


def learned() -> Workload:
    return Workload("learned: build workload, MLP 27-64-64-2 search window",
                    barrel(17), GenSettings(seed=SEED_BASE + 5, noise_lo=0.2, noise_hi=0.2), 1, 20000)


BARREL, DISK = 0, 1


@dataclass
class Detector:
    """General detector (section 4.1): barrel cylinders and endcap disks in
    the order a track from the origin meets them (barrel layers outwards,
    then the disks of each side outwards).  pos: average radius (barrel) or z
    of the average plane (disk); lo, hi: active extent in z (barrel) or r
    (disk); dmod: module offset from the average surface (modules of even
    phi sector at +dmod, odd at -dmod; n_mod sectors)."""
    kind: list
    pos: list
    lo: list
    hi: list
    dmod: list
    bz: float = f32(3.8)
    x_over_x0: float = f32(0.02)
    mass: float = f32(0.13957)
    beam_sigma: float = f32(0.01)
    n_mod: int = 24
    n_seed_layers: int = 3

    def __post_init__(self):
        for k in ("pos", "lo", "hi", "dmod"):
            setattr(self, k, [f32(v) for v in getattr(self, k)])
        self.kind = [int(v) for v in self.kind]
        self.bz, self.x_over_x0, self.mass = f32(self.bz), f32(self.x_over_x0), f32(self.mass)
        self.beam_sigma = f32(self.beam_sigma)

    @property
    def n_layers(self) -> int:
        return len(self.kind)

    def seed_geometry(self) -> Geometry:
        """The barrel of the seed layers (exact cylinders), for the seed
        convention."""
        ns = self.n_seed_layers
        assert all(k == BARREL for k in self.kind[:ns]) and all(d == 0 for d in self.dmod[:ns])
        zh = max(max(abs(v) for v in self.lo[:ns]), max(abs(v) for v in self.hi[:ns]))
        return Geometry(n_layers=ns, r=list(self.pos[:ns]), z_half=zh, bz=self.bz, x_over_x0=self.x_over_x0,
                        mass=self.mass, beam_sigma=self.beam_sigma)

    def replace(self, **kw) -> "Detector":
        return dataclasses.replace(self, **kw)


def cylinder_with_lids(dmod_barrel=0.5, dmod_disk=1.0, **kw) -> Detector:
    """Ten barrel layers at r = 4, 8, .., 40 cm (the three seed layers over
    |z| <= 100 cm, the others over |z| <= 50 cm, their modules 0.5 cm off the
    average radius) closed by seven disks on each side at |z| = 55 .. 112 cm
    covering 14 <= r <= 42 cm (modules 1 cm off the average z)."""
    zd = [55.0, 62.0, 70.0, 79.0, 89.0, 100.0, 112.0]
    kind = [BARREL] * 10 + [DISK] * 14
    pos = [4.0 * (i + 1) for i in range(10)] + zd + [-z for z in zd]
    lo = [-100.0] * 3 + [-50.0] * 7 + [14.0] * 14
    hi = [100.0] * 3 + [50.0] * 7 + [42.0] * 14
    dmod = [0.0] * 3 + [dmod_barrel] * 7 + [dmod_disk] * 14
    return Detector(kind, pos, lo, hi, dmod, **kw)


@dataclass
class DetWorkload:
    name: str
    detector: Detector
    gen: GenSettings
    n_events: int
    n_tracks: int
    cuts: BuildCuts = field(default_factory=BuildCuts)


def lids() -> DetWorkload:
    """Building and fitting in the cylinder with lids with displaced modules
    (two-step propagation): 20 000 tracks with |eta| <= 2 + 20 % noise per
    layer, 63 phi x 16 (z or r) bins per layer."""
    return DetWorkload("lids: 1 event x 20000 tracks |eta|<=2 + 20% noise/layer, 10 barrel layers + 2x7 disks, "
                       "modules off the average surface, 63x16 bins, cap 6, chi2<30, 1 hole",
                       cylinder_with_lids(), GenSettings(seed=SEED_BASE + 6, eta_max=2.0, noise_lo=0.2, noise_hi=0.2),
                       1, 20000)


def lids_fit() -> DetWorkload:
    """Fit at scale in the cylinder with lids: 50 events x 20 000 tracks."""
    return DetWorkload("lids_fit: 50 events x 20000 tracks |eta|<=2, 10 barrel layers + 2x7 disks, displaced modules",
                       cylinder_with_lids(), GenSettings(seed=SEED_BASE + 7, eta_max=2.0), 50, 20000)


ALL = {"fit_small": fit_small, "fit_scale": fit_scale, "build": build, "batch": batch, "learned": learned}
DETECTOR_WORKLOADS = {"lids": lids, "lids_fit": lids_fit}
