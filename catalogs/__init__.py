"""Seeded synthetic catalogs shaped like the paper's survey workloads.

This module is shared by the CPU oracle's tests and by the GPU path's tests and
benchmark. It only draws point positions: it holds none of the pair-counting
arithmetic (no separations, no binning, no estimators).

The paper measures on a MICE light-cone subset, on 600 PTHalo mocks and on a
log-normal mock (Sec. 4, Table 2, Figs. 5-6). None of those datasets is used
here; the catalogs below are seeded synthetic stand-ins with the same geometry,
sizes and kind of clustering.

Every generator takes explicit sizes so that the tests can draw small versions
of the same shapes. Random numbers come from numpy's ``Generator(PCG64(seed))``;
each catalog is shuffled so that input order carries no spatial structure.
Seeds follow ``1000 * w + role``, with w numbering the workload (1 periodic
uniform box, 2 clustered open box, 3 sigma-pi light cone, 4 angular cap,
5 batched mocks, 6 the Table 2 light-cone subset) and role 1 data, 2 randoms,
3 blob centres, 100+k mock k, 500 jackknife base.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Catalog", "rng", "uniform_box", "gaussian_blobs", "sky_cap_lightcone",
    "comoving_distance_table", "cap_uniform", "cap_blobs", "mock_sizes",
    "mixed_periodic", "periodic_uniform_2e4", "clustered_box_1e6", "lightcone_3e6",
    "angular_cap_1e7", "batched_mocks_256", "lightcone_box", "table2", "unit_vectors",
    "sha256_of",
]


@dataclass
class Catalog:
    """SoA float64 positions (3-D comoving, or unit vectors on the sphere)."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray

    def __len__(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx) -> "Catalog":
        return Catalog(np.ascontiguousarray(self.x[idx]),
                       np.ascontiguousarray(self.y[idx]),
                       np.ascontiguousarray(self.z[idx]))

    def head(self, n: int) -> "Catalog":
        return self.subset(slice(0, n))

    def stacked(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)

    @staticmethod
    def from_xyz(xyz: np.ndarray) -> "Catalog":
        xyz = np.asarray(xyz, dtype=np.float64)
        return Catalog(np.ascontiguousarray(xyz[:, 0]),
                       np.ascontiguousarray(xyz[:, 1]),
                       np.ascontiguousarray(xyz[:, 2]))


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _shuffled(g: np.random.Generator, xyz: np.ndarray) -> Catalog:
    perm = g.permutation(xyz.shape[0])
    return Catalog.from_xyz(xyz[perm])


def sha256_of(cat: Catalog) -> str:
    h = hashlib.sha256()
    for a in (cat.x, cat.y, cat.z):
        h.update(np.ascontiguousarray(a, dtype="<f8").tobytes())
    return h.hexdigest()


# ----------------------------------------------------------------------------
# 3-D boxes
# ----------------------------------------------------------------------------
def uniform_box(n: int, box: float, seed: int) -> Catalog:
    """n points uniform in [0, box)^3."""
    g = rng(seed)
    xyz = g.random((n, 3)) * box
    xyz = np.where(xyz >= box, np.nextafter(box, 0.0), xyz)
    return _shuffled(g, xyz)


def gaussian_blobs(n_centres: int, per_blob: int, sigma: float, box: float,
                   seed: int, centre_seed: int, wrap: bool) -> Catalog:
    """Blobs of ``per_blob`` points ~ N(c, sigma^2 I3) around centres uniform in
    [0, box)^3. With ``wrap`` the points are folded back into the periodic box,
    otherwise they are left where they fall (the catalog's bounding box then
    comes from the data)."""
    gc = rng(centre_seed)
    centres = gc.random((n_centres, 3)) * box
    g = rng(seed)
    off = g.normal(0.0, sigma, (n_centres, per_blob, 3))
    xyz = (centres[:, None, :] + off).reshape(-1, 3)
    if wrap:
        xyz = np.mod(xyz, box)
        xyz = np.where(xyz >= box, 0.0, xyz)
    return _shuffled(g, xyz)


# ----------------------------------------------------------------------------
# Light cone (sigma-pi workload)
# ----------------------------------------------------------------------------
C_OVER_H0 = 2997.92458  # Mpc/h


def comoving_distance_table(omega_m: float = 0.3, zmax: float = 3.0,
                            dz: float = 1e-4):
    """Trapezoid table of chi(z) = (c/H0) int_0^z dz'/E(z'), flat LCDM,
    E = sqrt(Om (1+z)^3 + 1 - Om). Used only to place synthetic galaxies."""
    zs = np.arange(0.0, zmax + dz / 2, dz)
    inv_e = 1.0 / np.sqrt(omega_m * (1.0 + zs) ** 3 + (1.0 - omega_m))
    chi = np.concatenate([[0.0], np.cumsum(0.5 * (inv_e[1:] + inv_e[:-1]) * dz)])
    return zs, C_OVER_H0 * chi


def sky_cap_lightcone(n: int, seed: int, ra_max_deg: float = 60.0,
                      dec_max_deg: float = 30.0, z_mean: float = 0.6,
                      z_sd: float = 0.15, z_min: float = 0.01) -> Catalog:
    """Points uniform on the sphere within RA in [0, ra_max], Dec in
    [0, dec_max], with a Gaussian n(z) (redrawn below z_min), placed at the
    flat-LCDM (Om=0.3) comoving distance. Observer at the origin."""
    g = rng(seed)
    ra = np.deg2rad(g.random(n) * ra_max_deg)
    sin_dec = g.random(n) * np.sin(np.deg2rad(dec_max_deg))
    z = g.normal(z_mean, z_sd, n)
    bad = z <= z_min
    while np.any(bad):
        z[bad] = g.normal(z_mean, z_sd, int(bad.sum()))
        bad = z <= z_min
    zs, chi_tab = comoving_distance_table()
    chi = np.interp(z, zs, chi_tab)
    cos_dec = np.sqrt(1.0 - sin_dec * sin_dec)
    xyz = np.stack([chi * cos_dec * np.cos(ra), chi * cos_dec * np.sin(ra),
                    chi * sin_dec], axis=1)
    return _shuffled(g, xyz)


def lightcone_box(n: int, seed: int, ra_max_deg: float = 18.0, dec_max_deg: float = 18.0,
                  z_lo: float = 0.5, z_hi: float = 0.6) -> Catalog:
    """Points uniform in comoving volume within RA in [0, ra_max], Dec in
    [0, dec_max] and redshift in [z_lo, z_hi] (flat LCDM, Om=0.3), observer
    at the origin: the shape of the light-cone subset the paper times its
    Table 2 on."""
    g = rng(seed)
    ra = np.deg2rad(g.random(n) * ra_max_deg)
    sin_dec = g.random(n) * np.sin(np.deg2rad(dec_max_deg))
    zs, chi_tab = comoving_distance_table()
    c0, c1 = np.interp([z_lo, z_hi], zs, chi_tab)
    chi = np.cbrt(c0 ** 3 + g.random(n) * (c1 ** 3 - c0 ** 3))
    cos_dec = np.sqrt(1.0 - sin_dec * sin_dec)
    xyz = np.stack([chi * cos_dec * np.cos(ra), chi * cos_dec * np.sin(ra),
                    chi * sin_dec], axis=1)
    return _shuffled(g, xyz)


def table2(n: int = 300_000):
    """Data and random catalogs of the Table 2 shape (about 3e5 points each).
    Returns (data, randoms) as 3-D positions; normalise them for angles."""
    return lightcone_box(n, seed=6001), lightcone_box(n, seed=6002)


def unit_vectors(cat: Catalog) -> Catalog:
    """The directions of a catalog's positions (observer at the origin)."""
    xyz = cat.stacked()
    return Catalog.from_xyz(xyz / np.linalg.norm(xyz, axis=1, keepdims=True))


# ----------------------------------------------------------------------------
# Unit vectors in a spherical cap (angular workload)
# ----------------------------------------------------------------------------
def _radec_to_vec(ra, dec):
    cd = np.cos(dec)
    return np.stack([cd * np.cos(ra), cd * np.sin(ra), np.sin(dec)], axis=-1)


def _cap_frame(ra0_deg: float, dec0_deg: float):
    ra0, dec0 = np.deg2rad(ra0_deg), np.deg2rad(dec0_deg)
    c = _radec_to_vec(ra0, dec0)
    # east and north tangent vectors at the cap centre
    e = np.array([-np.sin(ra0), np.cos(ra0), 0.0])
    nvec = np.cross(c, e)
    return c, e, nvec


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def cap_uniform(n: int, half_angle_deg: float, ra0_deg: float, dec0_deg: float,
                seed: int) -> Catalog:
    """n unit vectors uniform on the sphere within ``half_angle`` of the centre."""
    g = rng(seed)
    c, e, nv = _cap_frame(ra0_deg, dec0_deg)
    cmin = np.cos(np.deg2rad(half_angle_deg))
    cos_t = 1.0 - g.random(n) * (1.0 - cmin)
    phi = g.random(n) * 2.0 * np.pi
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    v = (cos_t[:, None] * c[None, :] + (sin_t * np.cos(phi))[:, None] * e[None, :]
         + (sin_t * np.sin(phi))[:, None] * nv[None, :])
    return _shuffled(g, _unit(v))


def cap_blobs(n_centres: int, per_blob: int, sigma_deg: float,
              half_angle_deg: float, ra0_deg: float, dec0_deg: float,
              seed: int, centre_seed: int) -> Catalog:
    """Angular Gaussian blobs: centres uniform in the cap, each point offset in
    the tangent plane of its centre by N(0, sigma^2) per axis, renormalised."""
    cen = cap_uniform(n_centres, half_angle_deg, ra0_deg, dec0_deg, centre_seed).stacked()
    g = rng(seed)
    # tangent basis at every centre
    zhat = np.array([0.0, 0.0, 1.0])
    t1 = np.cross(zhat[None, :], cen)
    small = np.linalg.norm(t1, axis=1) < 1e-8
    t1[small] = np.array([1.0, 0.0, 0.0])
    t1 = _unit(t1)
    t2 = np.cross(cen, t1)
    s = np.deg2rad(sigma_deg)
    a = g.normal(0.0, s, (n_centres, per_blob))
    b = g.normal(0.0, s, (n_centres, per_blob))
    v = cen[:, None, :] + a[..., None] * t1[:, None, :] + b[..., None] * t2[:, None, :]
    return _shuffled(g, _unit(v.reshape(-1, 3)))


# ----------------------------------------------------------------------------
# Batched mocks (periodic box)
# ----------------------------------------------------------------------------
def mock_sizes(n_mocks: int, n_lo: float, n_hi: float, seed: int) -> np.ndarray:
    g = rng(seed)
    return np.rint(np.exp(g.uniform(np.log(n_lo), np.log(n_hi), n_mocks))).astype(np.int64)


def mixed_periodic(n: int, box: float, seed: int, blob_frac: float = 0.5,
                   per_blob: int = 100, sigma: float = 5.0) -> Catalog:
    """Half uniform points, half Gaussian blobs (wrapped) in a periodic box."""
    nb = int(round(n * blob_frac / per_blob))
    nu = n - nb * per_blob
    g = rng(seed)
    u = g.random((nu, 3)) * box
    centres = g.random((nb, 3)) * box
    off = g.normal(0.0, sigma, (nb, per_blob, 3))
    bl = (centres[:, None, :] + off).reshape(-1, 3)
    xyz = np.mod(np.concatenate([u, bl], axis=0), box)
    xyz = np.where(xyz >= box, 0.0, xyz)
    return _shuffled(g, xyz)


# ----------------------------------------------------------------------------
# The five workload shapes (scale factors give the small test versions)
# ----------------------------------------------------------------------------
def periodic_uniform_2e4(n: int = 20_000, box: float = 1000.0) -> Catalog:
    """Monopole in a periodic box: uniform points."""
    return uniform_box(n, box, seed=1001)


def clustered_box_1e6(n_centres: int = 10_000, per_blob: int = 100, n_rand: int = 2_000_000,
            box: float = 2000.0, sigma: float = 5.0):
    """r-mu workload: clustered data (Gaussian blobs, not wrapped) and uniform
    randoms in an open box. Returns (data, randoms)."""
    d = gaussian_blobs(n_centres, per_blob, sigma, box, seed=2001, centre_seed=2003, wrap=False)
    r = uniform_box(n_rand, box, seed=2002)
    return d, r


def lightcone_3e6(n_data: int = 3_000_000, n_rand: int = 6_000_000, ra_max_deg: float = 60.0,
            dec_max_deg: float = 30.0):
    """sigma-pi light-cone workload. Returns (data, randoms)."""
    d = sky_cap_lightcone(n_data, seed=3001, ra_max_deg=ra_max_deg, dec_max_deg=dec_max_deg)
    r = sky_cap_lightcone(n_rand, seed=3002, ra_max_deg=ra_max_deg, dec_max_deg=dec_max_deg)
    return d, r


CAP_HALF_ANGLE_DEG = 40.75   # about 5000 sq-deg
CAP_CENTRE = (180.0, 0.0)    # (RA, Dec) in degrees


def angular_cap_1e7(n_centres: int = 100_000, per_blob: int = 100, n_rand: int = 20_000_000,
            half_angle_deg: float = CAP_HALF_ANGLE_DEG, centre=CAP_CENTRE,
            sigma_deg: float = 0.05):
    """Angular workload: clustered data and uniform randoms (unit vectors) in a
    spherical cap. Returns (data, randoms)."""
    d = cap_blobs(n_centres, per_blob, sigma_deg, half_angle_deg, centre[0], centre[1],
                  seed=4001, centre_seed=4003)
    r = cap_uniform(n_rand, half_angle_deg, centre[0], centre[1], seed=4002)
    return d, r


def batched_mocks_256(n_mocks: int = 256, n_lo: float = 2e4, n_hi: float = 5e5,
            jk_base: int = 1_000_000, box: float = 1000.0):
    """Batched mocks: sizes log-uniform in [n_lo, n_hi], half uniform half blobs,
    periodic; plus one jackknife base catalog and its 10x10 (x, y) column region
    labels. Returns (mocks, base, region_of_point)."""
    sizes = mock_sizes(n_mocks, n_lo, n_hi, seed=5099)
    mocks = [mixed_periodic(int(s), box, seed=5100 + k) for k, s in enumerate(sizes)]
    base = mixed_periodic(jk_base, box, seed=5500)
    ix = np.minimum((base.x * (10.0 / box)).astype(np.int64), 9)
    iy = np.minimum((base.y * (10.0 / box)).astype(np.int64), 9)
    region = (iy * 10 + ix).astype(np.int32)
    return mocks, base, region
