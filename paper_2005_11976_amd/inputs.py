"""Seeded synthetic inputs for the cylindrical-grid cone-beam path.

This module only *describes* scans: grid extents, circular trajectories in the
stage frame, rigid poses, phantom volumes painted on the cylindrical grid,
voxel-weight maps and Poisson counts.  It holds none of the method's
arithmetic (no ray tracing, no projection, no reconstruction), so both the
FP64 oracle and the HIP path can take their inputs from here without sharing
any computational code.

Conventions (the paper leaves them open; these are the readings used):
  * grid (Sec. 2, Eq. 2): r in [r_min, r_max], h in [h_min, h_max] about the
    object origin, theta sectors of width 2*pi/N_theta starting at theta0;
    volumes are C-ordered (N_h, N_theta, N_r), r fastest.
  * pose (Sec. 2, Eq. 1): X' = R X + T maps stage coordinates to the object
    frame; R = Rz(alpha) Rx(beta) Rz(gamma) (intrinsic zxz Euler angles).
    An object whose centre sits at c in the stage frame has T = -R c.
  * trajectory (Sec. 2.1, Table 1): circular, in the z = 0 plane, rotating
    counter-clockwise about +z; one 12-vector per view: source, detector
    centre, pixel step along a row (u), pixel step along a column (v).
  * attenuation: mu = density * 0.02 per mm.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

MU_PER_DENSITY = 0.02  # mm^-1 per unit density


@dataclasses.dataclass(frozen=True)
class Grid:
    """Cylindrical voxel grid (Sec. 2, Eq. 2): N_h x N_theta x N_r ring sectors."""
    n_h: int
    n_theta: int
    n_r: int
    r_min: float
    r_max: float
    h_min: float
    h_max: float
    theta0: float = 0.0

    @property
    def shape(self):
        return (self.n_h, self.n_theta, self.n_r)

    @property
    def n_vox(self):
        return self.n_h * self.n_theta * self.n_r


@dataclasses.dataclass(frozen=True)
class Scan:
    """A scan description: grid, stage-frame views, detector size and pose."""
    grid: Grid
    views: np.ndarray          # (n_views, 12) float64, stage frame
    det_rows: int
    det_cols: int
    R: np.ndarray              # (3, 3) float64
    T: np.ndarray              # (3,) float64

    @property
    def n_views(self):
        return int(self.views.shape[0])

    @property
    def proj_shape(self):
        return (self.n_views, self.det_rows, self.det_cols)


# --------------------------------------------------------------------------
# trajectories and poses
# --------------------------------------------------------------------------

def _rz(phi):
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rx(phi):
    c, s = math.cos(phi), math.sin(phi)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def circular_views(n_views, sod, sdd, pitch_u, pitch_v=None, arc=2 * math.pi,
                   endpoint=False, phi0=0.0):
    """Circular cone-beam trajectory, one 12-vector per view (stage frame).

    Source S_k = Rz(phi_k)(-SOD,0,0), detector centre D_k = Rz(phi_k)(SDD-SOD,0,0),
    u step Rz(phi_k)(0,p_u,0), v step (0,0,p_v).  With endpoint=False the views
    are phi_k = phi0 + arc*k/N (a full circle without a duplicate end view);
    with endpoint=True, phi_k = phi0 + arc*k/(N-1) (Table 1's 21 views over 200 deg).
    """
    pitch_v = pitch_u if pitch_v is None else pitch_v
    out = np.zeros((n_views, 12), dtype=np.float64)
    for k in range(n_views):
        if endpoint and n_views > 1:
            phi = phi0 + arc * k / (n_views - 1)
        else:
            phi = phi0 + arc * k / n_views
        Rz = _rz(phi)
        out[k, 0:3] = Rz @ np.array([-sod, 0.0, 0.0])
        out[k, 3:6] = Rz @ np.array([sdd - sod, 0.0, 0.0])
        out[k, 6:9] = Rz @ np.array([0.0, pitch_u, 0.0])
        out[k, 9:12] = np.array([0.0, 0.0, pitch_v])
    return out


def euler_zxz(alpha, beta, gamma):
    """R = Rz(alpha) Rx(beta) Rz(gamma) from intrinsic zxz Euler angles (Sec. 2, Eq. 1)."""
    return _rz(alpha) @ _rx(beta) @ _rz(gamma)


def pose_from(alpha, beta, gamma, centre):
    """(R, T) with X' = R X + T, for an object centred at `centre` (stage frame)."""
    R = euler_zxz(alpha, beta, gamma)
    T = -R @ np.asarray(centre, dtype=np.float64)
    return R, T


def identity_pose():
    return np.eye(3), np.zeros(3)


def random_pose(seed, max_tilt_deg=5.0, max_shift=2.0):
    """Seeded pose: beta ~ U[0, max_tilt], alpha, gamma ~ U[0, 2pi), shift with a
    uniform direction and |shift| ~ U[0, max_shift] mm."""
    rng = np.random.default_rng(seed)
    alpha = rng.uniform(0.0, 2 * math.pi)
    beta = math.radians(rng.uniform(0.0, max_tilt_deg))
    gamma = rng.uniform(0.0, 2 * math.pi)
    v = rng.normal(size=3)
    v /= np.linalg.norm(v)
    shift = v * rng.uniform(0.0, max_shift)
    R, T = pose_from(alpha, beta, gamma, shift)
    return R, T, dict(alpha=alpha, beta=beta, gamma=gamma, shift=shift)


# --------------------------------------------------------------------------
# phantoms painted on the grid (all voxel-aligned)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Phantom:
    truth: np.ndarray            # volume the data are simulated from (mu, 1/mm)
    prior: np.ndarray            # prior volume (with the removed component present)
    weights: np.ndarray          # voxel weight map
    annuli: list                 # (ih0, ih1, ir0, ir1, mu) painted in order
    blocks: list                 # (ih0, ih1, it0, it1, ir0, ir1, mu) ring-sector inclusions
    removed: Optional[int]       # index into blocks of the inclusion missing from `truth`
    ring: tuple                  # (ir0, ir1) radial band with the high weight


def coaxial_annuli_phantom(grid: Grid, densities):
    """Config-1 phantom: len(densities) annuli splitting the rings evenly, full height."""
    nb = len(densities)
    vol = np.zeros(grid.shape, dtype=np.float64)
    annuli = []
    for i, d in enumerate(densities):
        ir0 = i * grid.n_r // nb
        ir1 = (i + 1) * grid.n_r // nb
        mu = float(d) * MU_PER_DENSITY
        vol[:, :, ir0:ir1] = mu
        annuli.append((0, grid.n_h, ir0, ir1, mu))
    return vol, annuli


def tiny_phantom(grid: Grid, seed: int):
    rng = np.random.default_rng(seed)
    dens = rng.uniform(0.0, 1.0, size=4)
    vol, annuli = coaxial_annuli_phantom(grid, dens)
    return Phantom(truth=vol, prior=np.zeros_like(vol), weights=np.ones_like(vol),
                   annuli=annuli, blocks=[], removed=None, ring=(0, grid.n_r))


def industrial_phantom(grid: Grid, seed: int, n_annuli=6, n_incl=8,
                       w_ring=1.0, w_else=0.25):
    """Synthetic industrial part: `n_annuli` coaxial voxel-aligned cylinders or
    annuli (seeded radial and axial bounds, painted in order, density U[0.2,1]),
    and `n_incl` ring-sector inclusions inside the radial band of one component
    (theta width 8-40 sectors and h extent 16-64 slabs at 720 x 256, scaled with
    the grid).  One seeded inclusion is missing from the truth; the prior has it.
    Voxel weights: w_ring inside that band, w_else elsewhere."""
    rng = np.random.default_rng(seed)
    nh, nt, nr = grid.shape
    vol = np.zeros(grid.shape, dtype=np.float64)
    annuli = []
    # component 0: the body, all rings over most of the height
    h_lo = int(round(nh * rng.uniform(0.02, 0.08)))
    h_hi = nh - int(round(nh * rng.uniform(0.02, 0.08)))
    comps = [(h_lo, h_hi, 0, nr)]
    for _ in range(n_annuli - 1):
        ir0 = int(rng.integers(0, nr - nr // 8))
        ir1 = int(rng.integers(ir0 + max(1, nr // 16), nr + 1))
        ih0 = int(rng.integers(h_lo, h_hi - nh // 8))
        ih1 = int(rng.integers(ih0 + max(1, nh // 16), h_hi + 1))
        comps.append((ih0, ih1, ir0, ir1))
    for (ih0, ih1, ir0, ir1) in comps:
        mu = float(rng.uniform(0.2, 1.0)) * MU_PER_DENSITY
        vol[ih0:ih1, :, ir0:ir1] = mu
        annuli.append((ih0, ih1, ir0, ir1, mu))
    # the inclusion ring = radial band of one of the annular components
    ring_comp = comps[int(rng.integers(1, len(comps)))]
    r0, r1 = ring_comp[2], ring_comp[3]
    ring = (r0, r1)
    th_scale = nt / 720.0
    h_scale = nh / 256.0
    blocks = []
    for _ in range(n_incl):
        tw = max(1, int(round(rng.integers(8, 41) * th_scale)))
        hw = max(1, int(round(rng.integers(16, 65) * h_scale)))
        hw = min(hw, nh)
        tw = min(tw, nt)
        it0 = int(rng.integers(0, nt))
        ih0 = int(rng.integers(0, nh - hw + 1))
        rw = max(1, (r1 - r0) // 2)
        ir0 = int(rng.integers(r0, max(r0 + 1, r1 - rw + 1)))
        ir1 = min(r1, ir0 + rw)
        mu = float(rng.uniform(0.2, 1.0)) * MU_PER_DENSITY
        blocks.append((ih0, ih0 + hw, it0, it0 + tw, ir0, ir1, mu))
    removed = int(rng.integers(0, n_incl)) if n_incl else None
    prior = vol.copy()
    truth = vol.copy()
    for bi, (ih0, ih1, it0, it1, ir0, ir1, mu) in enumerate(blocks):
        idx_t = np.arange(it0, it1) % nt
        prior[ih0:ih1, idx_t, ir0:ir1] = mu
        if bi != removed:
            truth[ih0:ih1, idx_t, ir0:ir1] = mu
    weights = np.full(grid.shape, w_else, dtype=np.float64)
    weights[:, :, r0:r1] = w_ring
    return Phantom(truth=truth, prior=prior, weights=weights, annuli=annuli,
                   blocks=blocks, removed=removed, ring=ring)


def line_phantom(grid: Grid, kind: str, n_l: int, amplitude: float = MU_PER_DENSITY, background: float = 0.0):
    """Line phantoms of the MTF study (Sec. 2.3, Fig. 3): a cosine with n_l
    periods along theta (kind "azimuthal": every slice a Siemens star) or
    along r over [r_min, r_max] (kind "radial": concentric circles), between
    `background` and `background + amplitude`, constant along h.  Values are
    taken at the cell centres with the phase of the cell's lower edge, so that
    at the Nyquist rate (2 cells per period) the cells alternate between the
    two extremes (cell-centre phases would sample a cosine at its zeros
    there)."""
    nh, nt, nr = grid.shape
    if kind == "azimuthal":
        arg = 2.0 * math.pi * n_l * np.arange(nt) / nt
        prof = background + 0.5 * amplitude * (1.0 + np.cos(arg))
        vol = np.broadcast_to(prof[None, :, None], (nh, nt, nr))
    elif kind == "radial":
        arg = 2.0 * math.pi * n_l * np.arange(nr) / nr
        prof = background + 0.5 * amplitude * (1.0 + np.cos(arg))
        vol = np.broadcast_to(prof[None, None, :], (nh, nt, nr))
    else:
        raise ValueError("kind must be 'azimuthal' or 'radial'")
    return np.ascontiguousarray(vol, dtype=np.float64)


def interleaved_order(n_views):
    """A sweep order that visits far-apart views in turn: k_i = i s mod N with
    the step s nearest N (1 - 1/phi) (phi the golden ratio) that is coprime
    with N.  Consecutive SART updates then correct different directions,
    where the sequential order spends many updates on nearly the same one."""
    if n_views <= 2:
        return np.arange(n_views, dtype=np.int32)
    target = n_views * (1.0 - 2.0 / (1.0 + math.sqrt(5.0)))
    steps = sorted(range(1, n_views), key=lambda s_: (abs(s_ - target), s_))
    step = next(s_ for s_ in steps if math.gcd(s_, n_views) == 1)
    return ((np.arange(n_views, dtype=np.int64) * step) % n_views).astype(np.int32)


def mtf_setup(n_views, n_theta=512, fine=False):
    """Scan of the MTF study (Sec. 2.3 and 3.1): a 25 mm radius, 2.4 mm high
    sample on (S_h, S_theta, S_r) = (32, 1608, 256) (fine=True, the phantom
    grid) or (32, n_theta, 256) (the reconstruction grid, N_theta = 512 in the
    paper), n_views views over a full circle on a 2048 x 128 detector of
    0.05 mm pixels, SOD 200 mm, SDD 400 mm (the paper gives the detector
    size only: the sample fills its width and the cone stays within its
    height)."""
    nt = 1608 if fine else n_theta
    grid = Grid(32, nt, 256, 0.0, 25.0, -1.2, 1.2)
    views = circular_views(n_views, 200.0, 400.0, 0.05)
    return Scan(grid, views, 128, 2048, *identity_pose())


def poisson_line_integrals(p_clean, photons, seed):
    """Noisy line integrals from Poisson counts (Sec. 2.2, Eq. 6):
    I ~ Poisson(I0 exp(-p)),  p~ = -ln(max(I, 1) / I0)."""
    rng = np.random.default_rng(seed)
    counts = rng.poisson(photons * np.exp(-np.asarray(p_clean, dtype=np.float64)))
    return -np.log(np.maximum(counts, 1) / photons)


def uniform_vector(n, seed):
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=n)


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------

def config_tiny():
    """16x64x16 grid (r 10 mm, h 10 mm), SOD 100, SDD 200, 32 views over 360 deg,
    64 x 32 detector of 0.4 mm; 4 coaxial annuli; zero start; 10 iterations."""
    g = Grid(16, 64, 16, 0.0, 10.0, -5.0, 5.0)
    views = circular_views(32, 100.0, 200.0, 0.4)
    R, T = identity_pose()
    return dict(name="tiny_16x64x16", scan=Scan(g, views, 32, 64, R, T),
                seed=1001, n_iter=10, lam=0.5, weighted=False, from_prior=False)


def config_single():
    """256x720x128 grid (r 25 mm, h 50 mm), SOD 200, SDD 400, 120 views,
    512 x 512 detector of 0.2 mm; industrial phantom; weighted SART from the
    prior; 20 iterations."""
    g = Grid(256, 720, 128, 0.0, 25.0, -25.0, 25.0)
    views = circular_views(120, 200.0, 400.0, 0.2)
    R, T = identity_pose()
    return dict(name="single_256x720x128", scan=Scan(g, views, 512, 512, R, T),
                seed=1002, n_iter=20, lam=0.5, weighted=True, from_prior=True)


def config_posed():
    """512x1440x256 grid (r 40 mm, h 100 mm), SOD 300, SDD 600, 60 views,
    1024 cols x 768 rows of 0.15 mm; seeded pose (tilt <= 5 deg, shift <= 2 mm);
    Poisson noise at 1e4 photons; 30 weighted iterations from the prior."""
    g = Grid(512, 1440, 256, 0.0, 40.0, -50.0, 50.0)
    views = circular_views(60, 300.0, 600.0, 0.15)
    R, T, _ = random_pose(2003)
    return dict(name="posed_512x1440x256", scan=Scan(g, views, 768, 1024, R, T),
                seed=1003, n_iter=30, lam=0.5, weighted=True, from_prior=True,
                photons=1e4, noise_seed=3003)


def scaled_single(n_h=32, n_theta=96, n_r=16, n_views=24, det=64, posed_seed=None):
    """A reduced copy of the 256x720x128 scan (same extents and magnification,
    coarser grid and detector) small enough for full oracle SART runs."""
    g = Grid(n_h, n_theta, n_r, 0.0, 25.0, -25.0, 25.0)
    pitch = 0.2 * 512 / det
    views = circular_views(n_views, 200.0, 400.0, pitch)
    if posed_seed is None:
        R, T = identity_pose()
    else:
        R, T, _ = random_pose(posed_seed)
    return Scan(g, views, det, det, R, T)


# --------------------------------------------------------------------------
# the in-line serving stream (three object classes, Poisson arrivals)
# --------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class ScanClass:
    name: str
    grid: Grid
    views: np.ndarray
    det_rows: int
    det_cols: int
    phantom_seed: int

    def scan(self, R, T):
        return Scan(self.grid, self.views, self.det_rows, self.det_cols, R, T)


def serving_classes():
    """Classes A, B, C of the serving stream (SOD 200 mm, SDD 400 mm):
    A 128x360x64 (r 12.5, h 25 mm), 60 views of 256x256 at 0.2 mm;
    B 256x720x128 (r 25, h 50 mm), 90 views of 512x512 at 0.2 mm;
    C 384x1080x192 (r 37.5, h 75 mm), 120 views of 512 rows x 768 cols at 0.3 mm."""
    return [
        ScanClass("A", Grid(128, 360, 64, 0.0, 12.5, -12.5, 12.5), circular_views(60, 200.0, 400.0, 0.2),
                  256, 256, 1050),
        ScanClass("B", Grid(256, 720, 128, 0.0, 25.0, -25.0, 25.0), circular_views(90, 200.0, 400.0, 0.2),
                  512, 512, 1051),
        ScanClass("C", Grid(384, 1080, 192, 0.0, 37.5, -37.5, 37.5), circular_views(120, 200.0, 400.0, 0.3),
                  512, 768, 1052),
    ]


@dataclasses.dataclass(frozen=True)
class Request:
    rid: int
    cls: int
    arrival: float      # seconds from the start of the stream
    R: np.ndarray
    T: np.ndarray


def serving_requests(n, rate, n_classes=3, seed=6000, classes=None):
    """n requests with exponential inter-arrival times of mean 1/rate seconds
    (seed 6000), classes uniform over `classes` (default all n_classes), pose
    of request r from random_pose(5000 + r) (tilt <= 5 deg, shift <= 2 mm)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    pool = list(range(n_classes)) if classes is None else list(classes)
    kinds = rng.integers(0, len(pool), size=n)
    out = []
    for r in range(n):
        R, T, _ = random_pose(5000 + r)
        out.append(Request(r, pool[int(kinds[r])], float(arrivals[r]), R, T))
    return out
