"""The five seeded workloads (input recipes only).

cfg1  parity case: 64 antennas in a 5 km-radius disk, dec +45 deg, 2 h,
      60 samples, 1.4 GHz -> 2016 baselines x 60 = 120,960 rows; 200 components
      uniform in a 2 deg field; tree at J = 6.
cfg2  measured case: 256 antennas in a 20 km-radius disk, dec +30 deg, 8 h,
      256 samples, 1.4 GHz -> 32,640 x 256 = 8,355,840 rows; 2,000 components
      (70 % in 5 Gaussian blobs of sigma 0.1 deg, 30 % uniform over 4 deg);
      trees at J = 8, 9, 10.
cfg3  precision case: cfg2's layout with a 50 km-radius disk (baselines to
      ~100 km, w-term active), 10,000 components uniform over 3 deg.
cfg4  batched case: 64 channels (0.95-1.75 GHz) x 4 pointings; per instance
      2M-8M unflagged rows after 0-40 % random flagging, N_C log-uniform in
      [100, 20000], J uniform in 7..10.
cfg5  adjoint case: cfg2 tracks and model; a perturbed model plus complex
      noise (sigma 0.01 Jy) gives observed visibilities; residual image on the
      level-9 pixels within 4 deg of the phase centre.
sweep tree-route run-time sweep: a 27-antenna one-hour, one-second track
      (1,263,600 rows), 10-140 distinct components, J = 12-25.
clean7 the clean loop's wide-field simulation: the same array at 10 MHz for
      2,016 s (707,616 rows), seven 1 Jy sources, a 256 x 256 image over
      42 deg 40'; clean_small is its parity case (8,424 rows, 40 x 40 pixels).

The phase centre of every config is at right ascension 12h, the
declination of its tracks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import models, tracks


@dataclass(frozen=True)
class TrackSpec:
    n_ant: int
    radius_m: float
    dec_deg: float
    duration_s: float
    n_t: int
    freq_hz: float
    seed: int
    ra_deg: float = 180.0

    @property
    def n_baselines(self) -> int:
        return self.n_ant * (self.n_ant - 1) // 2

    @property
    def n_vis(self) -> int:
        return self.n_baselines * self.n_t

    def uvw(self):
        return tracks.array_tracks(self.n_ant, self.radius_m, self.dec_deg,
                                   self.duration_s, self.n_t, self.freq_hz, self.seed)

    def uvw_rows(self, rows):
        bxyz = tracks.array_baselines_xyz(self.n_ant, self.radius_m, self.seed)
        return tracks.uvw_rows(bxyz, self.n_t, self.duration_s, self.dec_deg,
                               self.freq_hz, rows)


@dataclass(frozen=True)
class Workload:
    name: str
    track: TrackSpec
    model: str                      # "uniform" or "mixture"
    n_comp: int
    field_deg: float
    seed_model: int
    J: tuple = ()
    description: str = ""

    @property
    def ra_p(self) -> float:
        return math.radians(self.track.ra_deg)

    @property
    def dec_p(self) -> float:
        return math.radians(self.track.dec_deg)

    def components(self):
        rng = np.random.default_rng(self.seed_model)
        if self.model == "uniform":
            return models.uniform_components(self.n_comp, self.field_deg, rng)
        return models.blob_mixture_components(self.n_comp, 0.7, 5, 0.1, 3.0,
                                              self.field_deg, rng)


H = 3600.0

CFG1 = Workload("cfg1", TrackSpec(64, 5e3, 45.0, 2 * H, 60, 1.4e9, seed=101),
                "uniform", 200, 2.0, seed_model=102, J=(6,),
                description="direct FP64 parity, 120,960 vis x 200 comps")
CFG2 = Workload("cfg2", TrackSpec(256, 20e3, 30.0, 8 * H, 256, 1.4e9, seed=201),
                "mixture", 2000, 4.0, seed_model=202, J=(8, 9, 10),
                description="direct vs tree FP64, 8,355,840 vis x 2,000 comps")
CFG3 = Workload("cfg3", TrackSpec(256, 50e3, 30.0, 8 * H, 256, 1.4e9, seed=301),
                "uniform", 10_000, 3.0, seed_model=302,
                description="FP32-compensated vs FP64, 8,355,840 vis x 10,000 comps")
CFG5_NOISE_SIGMA = 0.01
CFG5_J = 9
CFG5_DISK_RADIUS_DEG = 4.0
CFG5_SEED_PERTURB = 502
CFG5_SEED_NOISE = 503

WORKLOADS = {w.name: w for w in (CFG1, CFG2, CFG3)}

# Run-time sweep of the tree route (section 3.6.1): a JVLA-like one-hour track
# at one-second sampling, 27 antennas -> 351 baselines x 3600 = 1,263,600 rows
# (C-configuration extent, the 10 MHz, dec +45 deg simulation the sweep used);
# distinct components uniform over a 20 deg field.
SWEEP_TRACK = TrackSpec(27, 1.7e3, 45.0, 1 * H, 3600, 1.0e7, seed=601)
SWEEP_FIELD_DEG = 20.0
SWEEP_SEED_MODEL = 602


def sweep_components(n_distinct: int, seed: int = SWEEP_SEED_MODEL):
    """n_distinct components uniform over the sweep field, lognormal fluxes."""
    rng = np.random.default_rng(seed + n_distinct)
    return models.uniform_components(n_distinct, SWEEP_FIELD_DEG, rng)


# Clean loop (sections 2.2, 3.5, 3.6): the wide-field seven-source simulation.
# A 27-antenna C-configuration-like array (1.7 km radius), 10 MHz, dec +45 deg,
# 2,016 s at one-second sampling -> 351 x 2016 = 707,616 rows; seven compact
# 1 Jy sources uniform within a 30 deg field; complex noise of sigma 0.01 Jy;
# a 256 x 256 image grid over 42 deg 40'.
@dataclass(frozen=True)
class CleanSpec:
    track: TrackSpec
    n_pix: int                 # image is n_pix x n_pix
    fov_deg: float             # full width of the image in direction cosines (small angle)
    source_field_deg: float
    J: int
    gain: float
    minor_iter: int            # Hogbom iterations per major cycle
    n_major: int
    seed_model: int
    seed_noise: int
    noise_sigma: float = 0.01
    n_sources: int = 7

    @property
    def ra_p(self) -> float:
        return math.radians(self.track.ra_deg)

    @property
    def dec_p(self) -> float:
        return math.radians(self.track.dec_deg)

    @property
    def cell(self) -> float:
        return math.radians(self.fov_deg) / self.n_pix

    def sources(self):
        """(l, m, flux): n_sources 1 Jy sources uniform over source_field_deg."""
        rng = np.random.default_rng(self.seed_model)
        l, m, _ = models.uniform_components(self.n_sources, self.source_field_deg, rng)
        return l, m, np.ones(self.n_sources)

    def noise(self):
        rng = np.random.default_rng(self.seed_noise)
        return models.complex_noise(self.track.n_vis, self.noise_sigma, rng)


# J = 11: sphere pixels of 0.057 deg oversample the 0.167 deg image pixels
# about threefold (the section 3.5 rule asks for at least twofold).
CLEAN7 = CleanSpec(TrackSpec(27, 1.7e3, 45.0, 2016.0, 2016, 1.0e7, seed=701), 256,
                   42.0 + 40.0 / 60.0, 30.0, J=11, gain=0.1, minor_iter=300, n_major=2,
                   seed_model=702, seed_noise=703)
# The same array on a short track and a small grid: the parity case.
CLEAN_SMALL = CleanSpec(TrackSpec(27, 1.7e3, 45.0, 2016.0, 24, 1.0e7, seed=711), 40,
                        4.0, 3.0, J=11, gain=0.1, minor_iter=60, n_major=2,
                        seed_model=712, seed_noise=713)


# Predictor comparison on the clean7 grid (section 3.6.1's 140 distinct
# components): components on random image pixels within the 30 deg source
# field, lognormal fluxes.
COMPARE_N_COMP = 140
COMPARE_SEED = 741


def clean7_grid_model(n: int = COMPARE_N_COMP, seed: int = COMPARE_SEED):
    """(pixel ids of the 256 x 256 clean7 grid, fluxes): distinct pixels."""
    S = CLEAN7
    rng = np.random.default_rng(seed)
    h = models.half_width(S.source_field_deg) / S.cell
    c = S.n_pix // 2
    pix = set()
    while len(pix) < n:
        ix, iy = (int(np.rint(rng.uniform(-h, h))) + c for _ in range(2))
        pix.add(iy * S.n_pix + ix)
    pix = np.array(sorted(pix), dtype=np.int64)
    return pix, models.lognormal_fluxes(n, rng)


def sample_rows(n_vis: int, n_sample: int, seed: int, tile: int = 256) -> np.ndarray:
    """Sorted row indices: the first and last `tile` rows plus a seeded random
    sample, so a sample spans several kernel tiles and the ragged tail."""
    rng = np.random.default_rng(seed)
    head = np.arange(min(tile, n_vis))
    tail = np.arange(max(0, n_vis - tile), n_vis)
    rnd = rng.choice(n_vis, size=min(n_sample, n_vis), replace=False)
    return np.unique(np.concatenate([head, tail, rnd])).astype(np.int64)


# ---------------------------------------------------------------- cfg4 ----
@dataclass(frozen=True)
class Instance:
    index: int
    channel_hz: float
    dec_deg: float
    n_target: int
    flag_frac: float
    n_t: int
    n_comp: int
    J: int
    seed: int


@dataclass
class BatchedWorkload:
    """64 channels x 4 pointings on cfg2's 256-antenna, 20 km array."""
    n_channels: int = 64
    f_lo: float = 0.95e9
    f_hi: float = 1.75e9
    decs: tuple = (30.0, 45.0, 60.0, 10.0)
    n_min: int = 2_000_000
    n_max: int = 8_000_000
    flag_max: float = 0.4
    nc_min: int = 100
    nc_max: int = 20_000
    J_range: tuple = (7, 10)
    seed: int = 401
    scale: float = 1.0                 # < 1 shrinks every instance (tests only)
    instances: list = field(default_factory=list)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        freqs = np.linspace(self.f_lo, self.f_hi, self.n_channels)
        n_bl = CFG2.track.n_baselines
        out = []
        i = 0
        for dec in self.decs:
            for f in freqs:
                n_target = int(rng.integers(self.n_min, self.n_max + 1) * self.scale)
                frac = float(rng.uniform(0.0, self.flag_max))
                n_t = max(1, math.ceil(n_target / (n_bl * (1.0 - frac))))
                nc = int(round(math.exp(rng.uniform(math.log(self.nc_min),
                                                    math.log(self.nc_max)))))
                J = int(rng.integers(self.J_range[0], self.J_range[1] + 1))
                out.append(Instance(i, float(f), float(dec), n_target, frac, n_t, nc, J,
                                    seed=int(self.seed * 1000 + i)))
                i += 1
        self.instances = out

    def instance_inputs(self, inst: Instance):
        """(u, v, w, l, m, flux) of one instance: the cfg2 array tracked for 8 h
        at the instance's pointing and frequency with n_t samples, rows flagged
        at random with the instance's fraction."""
        rng = np.random.default_rng(inst.seed)
        bxyz = tracks.array_baselines_xyz(CFG2.track.n_ant, CFG2.track.radius_m,
                                          CFG2.track.seed)
        Hs = tracks.hour_angles(8 * H, inst.n_t)
        u, v, w = tracks.uvw_from_baselines(bxyz, Hs, math.radians(inst.dec_deg),
                                            inst.channel_hz)
        keep = rng.random(u.shape[0]) >= inst.flag_frac
        l, m, flux = models.blob_mixture_components(inst.n_comp, 0.7, 5, 0.1, 3.0, 4.0, rng)
        return (np.ascontiguousarray(u[keep]), np.ascontiguousarray(v[keep]),
                np.ascontiguousarray(w[keep]), l, m, flux)

    def instance_rows_kept(self, inst: Instance):
        """Original (time-major) row index of every unflagged row, and the
        instance's components, drawn exactly as instance_inputs draws them."""
        rng = np.random.default_rng(inst.seed)
        n_rows = CFG2.track.n_baselines * inst.n_t
        keep = rng.random(n_rows) >= inst.flag_frac
        l, m, flux = models.blob_mixture_components(inst.n_comp, 0.7, 5, 0.1, 3.0, 4.0, rng)
        return np.nonzero(keep)[0].astype(np.int64), l, m, flux

    def instance_uvw_rows(self, inst: Instance, rows):
        """(u, v, w) of selected original rows, element by element on the host."""
        bxyz = tracks.array_baselines_xyz(CFG2.track.n_ant, CFG2.track.radius_m,
                                          CFG2.track.seed)
        return tracks.uvw_rows(bxyz, inst.n_t, 8 * H, inst.dec_deg, inst.channel_hz, rows)

    def instance_uvw_torch(self, inst: Instance, kept, device):
        """(u, v, w) of the kept rows as float64 tensors on `device`.  The same
        expressions as tracks.uvw_from_baselines in the same order, evaluated
        with torch element by element (sin and cos of the hour angles on the
        host), so each row equals the host generator's."""
        import torch
        bxyz = tracks.array_baselines_xyz(CFG2.track.n_ant, CFG2.track.radius_m,
                                          CFG2.track.seed)
        Hs = tracks.hour_angles(8 * H, inst.n_t)
        lam = tracks.C_LIGHT / inst.channel_hz
        dec = math.radians(inst.dec_deg)
        sd, cd = np.sin(dec), np.cos(dec)
        T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,  # noqa
                                      device=device)
        X, Y, Z = (T(bxyz[:, i])[None, :] for i in range(3))
        sH, cH = T(np.sin(Hs))[:, None], T(np.cos(Hs))[:, None]
        idx = torch.as_tensor(kept, device=device)
        out = []
        for expr in ("u", "v", "w"):
            if expr == "u":
                a = sH * X + cH * Y
            elif expr == "v":
                a = (-sd) * cH * X + (sd * sH) * Y + cd * Z
            else:
                a = (cd * cH) * X - (cd * sH) * Y + sd * Z
            a = a.reshape(-1).index_select(0, idx)
            out.append((a / torch.full_like(a, lam)).contiguous())
            del a
        return tuple(out)
