"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the pCMD method itself.  It only makes the
*data* the method consumes, as stand-ins for what the paper takes from outside
sources (stellar isochrones, instrument PSFs, observing set-ups) and for the
parameter points a sampler would propose:

* isochrone grids: per isochrone an age bin and a metallicity, per point an
  initial mass and absolute magnitudes in each band (the paper draws these from
  MIST isochrones, Sec. 2.2, which are not available here);
* PSF images: truncated Gaussians renormalised to unit sum (the paper uses
  Tiny Tim models, Sec. 2.2);
* observation set-ups: exposure times, zero-points, reddening coefficients;
* parameter vectors drawn from the priors of the mock tests (Sec. 3.1).

Every generator is deterministic given its arguments (and seed, where taken).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# ---------------------------------------------------------------------------
# isochrone grids
# ---------------------------------------------------------------------------


@dataclass
class IsoGrid:
    """A set of isochrones flattened into one entry list.

    iso_of_entry[E]     which isochrone each entry belongs to
    mass[E]             initial mass in solar masses, increasing inside an isochrone
    absmag[B][E]        absolute magnitude per band
    iso_log_age_lo/hi   edges (log10 yr) of the age bin each isochrone stands for
    iso_log_age         the isochrone's own age (log10 yr): bin midpoint
    iso_feh             [Fe/H] of each isochrone
    age_index, feh_index  position of each isochrone on the (age, [Fe/H]) grid
    """

    iso_of_entry: np.ndarray
    mass: np.ndarray
    absmag: np.ndarray
    iso_log_age_lo: np.ndarray
    iso_log_age_hi: np.ndarray
    iso_log_age: np.ndarray
    iso_feh: np.ndarray
    age_index: np.ndarray
    feh_index: np.ndarray
    age_edges: np.ndarray          # n_age + 1 edges, log10 yr
    feh_grid: np.ndarray           # n_feh values
    band_names: tuple = field(default_factory=tuple)

    @property
    def n_entries(self) -> int:
        return int(self.mass.shape[0])

    @property
    def n_bands(self) -> int:
        return int(self.absmag.shape[0])

    @property
    def n_iso(self) -> int:
        return int(self.iso_feh.shape[0])

    def subsample(self, stride: int) -> "IsoGrid":
        """Keep every `stride`-th mass point of each isochrone (always keeping
        the last point), like the paper's mass down-sampling hyper-parameter."""
        keep = []
        for k in range(self.n_iso):
            idx = np.nonzero(self.iso_of_entry == k)[0]
            sel = idx[::stride]
            if sel[-1] != idx[-1]:
                sel = np.concatenate([sel, idx[-1:]])
            keep.append(sel)
        keep = np.concatenate(keep)
        return IsoGrid(self.iso_of_entry[keep].copy(), self.mass[keep].copy(),
                       self.absmag[:, keep].copy(), self.iso_log_age_lo, self.iso_log_age_hi,
                       self.iso_log_age, self.iso_feh, self.age_index, self.feh_index,
                       self.age_edges, self.feh_grid, self.band_names)


def _luminosity_ms(m: np.ndarray) -> np.ndarray:
    """Textbook piecewise main-sequence mass-luminosity relation (L_sun)."""
    m = np.asarray(m, dtype=np.float64)
    return np.where(m < 0.43, 0.23 * m ** 2.3, np.where(m < 2.0, m ** 4.0, 1.4 * m ** 3.5))


def _colour_ms(m: np.ndarray) -> np.ndarray:
    return np.clip(1.2 - 0.9 * np.log10(m), -0.3, 2.0)


def _bands_from(mbol: np.ndarray, colour: np.ndarray, n_bands: int) -> np.ndarray:
    """Spread a bolometric magnitude over bands ordered blue to red.

    band 0 = mbol + c/2 (blue), band 1 = mbol - c/2 (red), band 2 = mbol - c (redder)."""
    offs = [0.5, -0.5, -1.0, -1.5][:n_bands]
    return np.stack([mbol + o * colour for o in offs])


def isochrone_ssp(n_pts: int = 500, m_lo: float = 0.1, m_hi: float = 20.0, n_bands: int = 2,
                  log_age: float = 9.0, feh: float = 0.0) -> IsoGrid:
    """One isochrone of `n_pts` masses log-spaced over [m_lo, m_hi] (a main
    sequence only; the 64x64 / 500-point small case)."""
    mass = np.geomspace(m_lo, m_hi, n_pts)
    mbol = 4.74 - 2.5 * np.log10(_luminosity_ms(mass))
    absmag = _bands_from(mbol, _colour_ms(mass), n_bands)
    one = np.zeros(1)
    return IsoGrid(np.zeros(n_pts, np.int32), mass, absmag,
                   one + log_age - 0.1, one + log_age + 0.1, one + log_age, one + feh,
                   np.zeros(1, np.int32), np.zeros(1, np.int32),
                   np.array([log_age - 0.1, log_age + 0.1]), np.array([feh]),
                   tuple(f"b{b}" for b in range(n_bands)))


def isochrone_grid(n_age: int = 7, feh_grid=(-0.75, -0.5, -0.25, 0.0, 0.25), n_pts: int = 1500,
                   n_bands: int = 3, log_age_min: float = 6.0, log_age_max: float = 10.2,
                   post_ms_frac: float = 0.15) -> IsoGrid:
    """Synthetic age x [Fe/H] grid of isochrones (stand-in for MIST tracks).

    Age bins are equal in log age between log_age_min and log_age_max; each
    isochrone sits at its bin midpoint.  Per isochrone: a main sequence of
    log-spaced masses from 0.1 Msun up to the turn-off mass
    M_TO = (t / 10 Gyr)^-0.4, then a post-main-sequence branch of the last
    `post_ms_frac` of the points over masses just above the turn-off that gets
    3..6 mag brighter and redder by 1.0 + 0.3 [Fe/H]; every colour is shifted
    by +0.3 [Fe/H]."""
    feh_grid = np.asarray(feh_grid, dtype=np.float64)
    edges = np.linspace(log_age_min, log_age_max, n_age + 1)
    n_post = int(round(post_ms_frac * n_pts))
    n_ms = n_pts - n_post
    iso_of, masses, mags = [], [], []
    lo, hi, mid, fe, ai, fi = [], [], [], [], [], []
    k = 0
    for a in range(n_age):
        la = 0.5 * (edges[a] + edges[a + 1])
        t_gyr = 10.0 ** la / 1e9
        m_to = min((t_gyr / 10.0) ** -0.4, 60.0)
        for f, feh in enumerate(feh_grid):
            m_ms = np.geomspace(0.1, m_to, n_ms)
            m_post = m_to * np.geomspace(1.0 + 1e-3, 1.08, n_post)
            mass = np.concatenate([m_ms, m_post])
            lum = _luminosity_ms(mass)
            mbol = 4.74 - 2.5 * np.log10(lum)
            col = _colour_ms(mass) + 0.3 * feh
            s = np.linspace(0.0, 1.0, n_post)
            mbol[n_ms:] = mbol[n_ms - 1] - (3.0 + 3.0 * s)
            col[n_ms:] = col[n_ms - 1] + (1.0 + 0.3 * feh) * (0.3 + 0.7 * s)
            iso_of.append(np.full(n_pts, k, np.int32))
            masses.append(mass)
            mags.append(_bands_from(mbol, col, n_bands))
            lo.append(edges[a]); hi.append(edges[a + 1]); mid.append(la); fe.append(feh)
            ai.append(a); fi.append(f)
            k += 1
    return IsoGrid(np.concatenate(iso_of), np.concatenate(masses), np.concatenate(mags, axis=1),
                   np.array(lo), np.array(hi), np.array(mid), np.array(fe),
                   np.array(ai, np.int32), np.array(fi, np.int32), edges, feh_grid,
                   tuple(f"b{b}" for b in range(n_bands)))


# ---------------------------------------------------------------------------
# PSFs and observation set-ups
# ---------------------------------------------------------------------------


def psf_gaussian(k: int, sigma: float) -> np.ndarray:
    """K x K truncated circular Gaussian, renormalised to unit sum in FP64 and
    stored FP32 (the same array is handed to every implementation)."""
    h = (k - 1) // 2
    y, x = np.mgrid[-h:h + 1, -h:h + 1].astype(np.float64)
    p = np.exp(-0.5 * (x * x + y * y) / (sigma * sigma))
    p /= p.sum()
    return p.astype(np.float32)


def psf_stack(k: int, sigmas) -> np.ndarray:
    return np.stack([psf_gaussian(k, s) for s in sigmas]).astype(np.float32)


def psf_gaussian_shifted(k: int, sigma: float, dy: float, dx: float) -> np.ndarray:
    """K x K truncated circular Gaussian centred (dy, dx) px off the kernel centre, renormalised
    to unit sum in FP64 and stored FP32."""
    h = (k - 1) // 2
    y, x = np.mgrid[-h:h + 1, -h:h + 1].astype(np.float64)
    p = np.exp(-0.5 * ((x - dx) ** 2 + (y - dy) ** 2) / (sigma * sigma))
    p /= p.sum()
    return p.astype(np.float32)


def psf_subpixel_stack(k: int, sigmas) -> np.ndarray:
    """[B][16][K][K]: per band the 4 x 4 grid of sub-pixel PSFs, region r = 4 ry + rx centred
    (ry / 4, rx / 4) px off the kernel centre (the paper's 4 x 4 sub-pixel model, Sec. 2.2)."""
    return np.stack([np.stack([psf_gaussian_shifted(k, s, ry / 4.0, rx / 4.0) for ry in range(4) for rx in range(4)])
                     for s in sigmas]).astype(np.float32)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------


@dataclass
class Obs:
    """Observation + nuisance set-up of one simulation (plain numbers)."""
    nim: int
    seed: int
    dmod: float
    dust_model: int = 0          # 0 none, 1 fixed screen, 2 log-normal screen
    dust_mu: float = -0.5        # log10 E(B-V) (median)
    dust_sigma: float = 0.2      # dex
    dust_frac: float = 0.5       # F_dust
    dust_R: tuple = (3.6, 1.9, 1.3)
    psf: np.ndarray | None = None  # [B][K][K] float32
    noise_model: int = 1         # 0 none, 1 Gaussian magnitude noise, 2 shot noise
    noise_sigma_mag: tuple = (0.02, 0.02, 0.02)
    exptime: tuple = (3620.0, 3235.0, 3000.0)
    zp: tuple = (26.0, 25.5, 25.0)
    sky: tuple = (0.0, 0.0, 0.0)
    sampler: int = 0             # 0 one count per (pixel, point); 1 block-skip superposition; 2 hybrid


@dataclass
class Model:
    """Physical model: which SFH / MDF form and its parameters."""
    sfh: str = "ssp"             # ssp | const | tau | dtau | nonparam
    log_npix: float = 2.0
    tau_gyr: float = 3.0
    ssp_age_index: int = 0
    log_sfh: tuple = ()          # nonparam: log10 stars per pixel per age bin
    mdf: str = "single"          # single | gauss
    feh_index: int = 0
    feh_mu: float = -0.25
    feh_sigma: float = 0.2
    mdf_prune: float = 0.01
    imf_alpha: float = 2.35
    imf: str = "salpeter"        # salpeter (power law, imf_alpha) | kroupa


def small_case(nim: int = 64, seed: int = 1):
    """64x64 image, 2 bands, one isochrone of 500 masses log-spaced 0.1-20 Msun,
    Salpeter weights at Npix = 100, no dust, 5x5 Gaussian PSF (sigma 1 px),
    Gaussian magnitude noise 0.02, distance modulus 25."""
    grid = isochrone_ssp(500, 0.1, 20.0, 2)
    model = Model(sfh="ssp", log_npix=2.0, mdf="single")
    obs = Obs(nim=nim, seed=seed, dmod=25.0, dust_model=0, psf=psf_stack(5, (1.0, 1.0)),
              noise_model=1, noise_sigma_mag=(0.02, 0.02), exptime=(3620.0, 3235.0),
              zp=(26.0, 25.5), sky=(0.0, 0.0), dust_R=(3.6, 1.9))
    return grid, model, obs


def headline_grid() -> IsoGrid:
    """7 log-age bins x 5 [Fe/H] points x 1500 masses = 52,500 entries, 3 bands."""
    return isochrone_grid(7, (-0.75, -0.5, -0.25, 0.0, 0.25), 1500, 3)


def draw_headline_params(seed: int, log_npix=None):
    """Parameters of one 256x256 evaluation, drawn from the mock-test priors:
    log Npix ~ U[2, 5], tau ~ U[0.1, 8] Gyr, mu_[Fe/H] ~ U[-0.5, 0.25],
    mu_dust ~ U[-1, 0] (sigma_dust 0.2 dex, F_dust 0.5), mu_d ~ U[24, 30]."""
    r = np.random.default_rng(np.random.SeedSequence([20190401, seed]))
    lnp = r.uniform(2.0, 5.0) if log_npix is None else float(log_npix)
    model = Model(sfh="tau", log_npix=lnp, tau_gyr=r.uniform(0.1, 8.0), mdf="gauss",
                  feh_mu=r.uniform(-0.5, 0.25), feh_sigma=0.2, mdf_prune=0.01)
    obs = Obs(nim=256, seed=seed, dmod=r.uniform(24.0, 30.0), dust_model=2,
              dust_mu=r.uniform(-1.0, 0.0), dust_sigma=0.2, dust_frac=0.5,
              dust_R=(3.6, 1.9, 1.3), psf=psf_stack(31, (1.6, 1.8, 2.0)), noise_model=2,
              exptime=(3620.0, 3235.0, 3000.0), zp=(26.0, 25.5, 25.0), sky=(0.0, 0.0, 0.0))
    return model, obs


def draw_large_params(seed: int):
    """Parameters of one 512x512 evaluation at Npix = 1e6 (most bright entries above the
    rejection threshold): the headline priors for SFH shape, metallicity, dust and distance,
    with 63x63 Gaussian PSFs (sigma = 3.2, 3.6, 4.0 px); used with a 200 x 200 Hess."""
    model, obs = draw_headline_params(seed, log_npix=6.0)
    obs.nim = 512
    obs.psf = psf_stack(63, (3.2, 3.6, 4.0))
    return model, obs


def hess_grid_from_median(mx: float, my: float, nx: int = 100, ny: int = 100, d: float = 0.05):
    """Hess origin: the data's median (colour, magnitude) floored to a multiple
    of the bin width, minus half the grid extent."""
    x0 = math.floor(mx / d) * d - (nx // 2) * d
    y0 = math.floor(my / d) * d - (ny // 2) * d
    return dict(x0=x0, dx=d, y0=y0, dy=d, nx=nx, ny=ny)


def batch_workload(n_jobs: int = 256, seed0: int = 0, nim_log2=(6.0, 9.0), entries=(5000, 52500), psf_k: int = 31,
                   grid: IsoGrid | None = None):
    """Uneven batch of parameter points: per job an image side 2^U[6, 9] rounded to a multiple of
    16, an isochrone set of U[5k, 52.5k] entries (mass points of the headline grid subsampled),
    and parameters drawn from the mock-test priors with seed `seed0 + j`.  Returns a list of
    (grid, model, obs) tuples; grids are shared between jobs with the same subsampling."""
    base = headline_grid() if grid is None else grid
    cache = {}
    out = []
    for j in range(n_jobs):
        r = np.random.default_rng(np.random.SeedSequence([4242, seed0 + j]))
        nim = int(round(2.0 ** r.uniform(*nim_log2) / 16.0)) * 16
        nim = max(nim, 16)
        e_target = r.uniform(*entries)
        stride = max(1, int(round(base.n_entries / e_target)))
        if stride not in cache:
            cache[stride] = base.subsample(stride)
        model, obs = draw_headline_params(seed0 + j)
        obs.nim = nim
        if psf_k != 31:
            obs.psf = psf_stack(psf_k, (1.6, 1.8, 2.0))
        out.append((cache[stride], model, obs))
    return out


def mlp_init(dims, seed: int = 0) -> np.ndarray:
    """Initial surrogate weights (packed per layer: W [out][in] then b [out]): uniform He-style
    weights, zero biases, FP32."""
    r = np.random.default_rng(seed)
    parts = []
    for l in range(len(dims) - 1):
        lim = math.sqrt(6.0 / dims[l])
        parts.append(r.uniform(-lim, lim, dims[l + 1] * dims[l]))
        parts.append(np.zeros(dims[l + 1]))
    return np.concatenate(parts).astype(np.float32)


SURROGATE_PARAM_NAMES = ("logSFH0", "logSFH1", "logSFH2", "logSFH3", "logSFH4", "logSFH5", "logSFH6",
                         "feh_mu", "feh_sigma", "dust_mu", "dust_sigma", "dmod")


def surrogate_truth() -> np.ndarray:
    """The 12-parameter vector of the mock data: the paper's fiducial-tau values (Sec. 3.1):
    tau = 3 Gyr SFH at Npix = 10^2 spread over the 7 age bins, mu_[Fe/H] = -0.25,
    sigma_[Fe/H] = 0.2, mu_dust = -0.5, sigma_dust = 0.1, mu_d = 26."""
    edges = headline_grid().age_edges
    T = 10.0 ** 10.2
    tau = 3e9
    t1 = T - 10.0 ** edges[1:]
    t2 = T - 10.0 ** edges[:-1]
    w = np.exp(-t1 / tau) - np.exp(-t2 / tau)
    log_sfh = np.log10(w / w.sum() * 100.0)
    return np.concatenate([log_sfh, [-0.25, 0.2, -0.5, 0.1, 26.0]])


def surrogate_box(center=None):
    """Parameter box of the surrogate's training draws and of the sampler's flat prior: log SFH
    bins +-0.5 dex around the truth, mu_[Fe/H] +-0.25, sigma_[Fe/H] in [0.1, 0.3],
    mu_dust +-0.25, sigma_dust in [0.05, 0.3], mu_d +-1."""
    c = surrogate_truth() if center is None else np.asarray(center, np.float64)
    lo = np.concatenate([c[:7] - 0.5, [c[7] - 0.25, 0.1, c[9] - 0.25, 0.05, c[11] - 1.0]])
    hi = np.concatenate([c[:7] + 0.5, [c[7] + 0.25, 0.3, c[9] + 0.25, 0.3, c[11] + 1.0]])
    return lo, hi


def surrogate_theta_draws(n: int, seed: int = 0, box=None):
    """n parameter vectors uniform in the surrogate box (12 parameters: log SFH of the 7 age bins
    in stars per pixel, mu_[Fe/H], sigma_[Fe/H], mu_dust, sigma_dust, mu_d)."""
    lo, hi = surrogate_box() if box is None else box
    r = np.random.default_rng(np.random.SeedSequence([777, seed]))
    return lo + (hi - lo) * r.uniform(size=(n, len(lo)))


def theta_to_model(th, seed: int, nim: int = 128):
    """(Model, Obs) of one 12-parameter vector on the headline grid and observation set-up."""
    th = np.asarray(th, dtype=np.float64)
    model = Model(sfh="nonparam", log_sfh=tuple(th[:7]), mdf="gauss", feh_mu=float(th[7]),
                  feh_sigma=float(th[8]), mdf_prune=0.01)
    obs = Obs(nim=nim, seed=seed, dmod=float(th[11]), dust_model=2, dust_mu=float(th[9]),
              dust_sigma=float(th[10]), dust_frac=0.5, dust_R=(3.6, 1.9, 1.3),
              psf=psf_stack(31, (1.6, 1.8, 2.0)), noise_model=2, exptime=(3620.0, 3235.0, 3000.0),
              zp=(26.0, 25.5, 25.0), sky=(0.0, 0.0, 0.0))
    return model, obs
