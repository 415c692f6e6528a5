"""Seeded synthetic networks: the only module shared by the solver and its checker.

It draws bond conductances for square (2D) and simple-cubic (3D) lattices in the
families the paper studies (Sec. II and Sec. VI): i.i.d. log-normal resistors,
fractional-Brownian-motion (FBM) correlated fields made by Fourier filtering of
white noise (Eq. 1, with the anisotropic form of Eq. 2), stratified layers, and
percolation dilution, either independent per bond (Sec. VI.A) or by removing the
smallest conductances (Sec. VI.B). It holds none of the flow computation: no
mask, no matrix, no solve.

Conventions (shared by every caller):

* A lattice of ``nx * ny * nz`` nodes (``nz == 1`` in 2D) is stored with x
  fastest: node ``i = x + nx * (y + ny * z)``; numpy arrays have shape
  ``(nz, ny, nx)`` (3D) or ``(ny, nx)`` (2D).
* Bond array ``g[k]`` has the node shape; ``g[k][i]`` is the conductance of the
  bond from node ``i`` to its neighbour ``i + e_k``. Entries whose neighbour
  lies past the lattice edge carry no bond and are set to 0. A removed
  (diluted) bond has conductance 0.
* Randomness: numpy ``PCG64``. Network ``i`` of a workload draws from
  ``SeedSequence(MASTER_SEED, spawn_key=(i,))`` (the i-th child of the master
  sequence); the field's normals are drawn first, then dilution uniforms.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

MASTER_SEED = 190803301


def rng_for(index: int, master: int = MASTER_SEED) -> np.random.Generator:
    """Generator of network ``index``: child ``index`` of the master seed sequence."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(master, spawn_key=(int(index),))))


# ----------------------------------------------------------------------------- lattices

@dataclass
class Network:
    """One synthetic network: lattice shape, flow axis and FP64 bond arrays."""

    dim: int
    nx: int
    ny: int
    nz: int
    g: List[np.ndarray]                      # dim arrays, node-shaped, float64, C-contiguous
    axis: int = 0
    meta: dict = field(default_factory=dict)
    periodic: bool = False                   # directions other than the flow axis wrap around

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def shape(self) -> Tuple[int, ...]:
        return (self.ny, self.nx) if self.dim == 2 else (self.nz, self.ny, self.nx)

    def with_axis(self, axis: int) -> "Network":
        return Network(self.dim, self.nx, self.ny, self.nz, self.g, axis, dict(self.meta), self.periodic)

    def with_periodic(self, periodic: bool = True) -> "Network":
        """Same bond arrays with periodic (or no-flow) side boundaries.

        The last-plane entries of the transverse bond arrays are the wrap
        bonds of a periodic network; the generators below draw them when
        called with ``periodic=True`` and zero them otherwise.
        """
        return Network(self.dim, self.nx, self.ny, self.nz, self.g, self.axis, dict(self.meta), bool(periodic))


def node_shape(dim: int, nx: int, ny: int, nz: int = 1) -> Tuple[int, ...]:
    if dim == 2:
        return (ny, nx)
    return (nz, ny, nx)


def clear_edge(a: np.ndarray, k: int) -> np.ndarray:
    """Copy of bond array ``a`` of direction k with its last-plane entries zeroed."""
    a = np.array(a, dtype=np.float64, copy=True, order="C")
    ax = a.ndim - 1 - k                      # numpy axis of lattice direction k (x is last)
    sl = [slice(None)] * a.ndim
    sl[ax] = -1
    a[tuple(sl)] = 0.0
    return a


def clear_edge_bonds(g: List[np.ndarray]) -> List[np.ndarray]:
    """Zero the entries of bond array k whose neighbour ``i + e_k`` is outside the lattice."""
    return [clear_edge(a, k) for k, a in enumerate(g)]


def edge_valid(dim: int, shape: Tuple[int, ...], k: int) -> np.ndarray:
    """Boolean node-shaped array: True where bond k from that node exists in the lattice."""
    m = np.ones(shape, dtype=bool)
    ax = dim - 1 - k
    sl = [slice(None)] * dim
    sl[ax] = -1
    m[tuple(sl)] = False
    return m


# ----------------------------------------------------------------------------- fields

def fbm_field(shape: Sequence[int], H: float, rng: np.random.Generator,
              beta: Optional[Sequence[float]] = None) -> np.ndarray:
    """Periodic FBM-correlated Gaussian field by Fourier filtering (Eqs. 1-2).

    White normals (one per grid point, drawn in C order) are transformed, each
    mode is scaled by the square root of the power spectrum
    ``S(k) = (sum_j beta_j k_j^2)^{-(H + d/2)}`` (d = number of grid axes; for
    d = 2 this is Eq. 1's exponent H + 1, and with ``beta`` Eq. 2's anisotropic
    form), the k = 0 mode is removed, and the real part of the inverse transform
    is standardised to mean 0 and standard deviation 1. ``beta`` lists the
    anisotropy factor of each numpy axis (default all 1).
    """
    shape = tuple(int(s) for s in shape)
    noise = rng.standard_normal(shape)
    return fbm_filter(noise, H, beta)


def fbm_filter(noise: np.ndarray, H: float, beta: Optional[Sequence[float]] = None) -> np.ndarray:
    """The filtering step of `fbm_field` on given white noise (see there)."""
    shape = noise.shape
    d = len(shape)
    spec = np.fft.fftn(noise)
    if beta is None:
        beta = [1.0] * d
    k2 = np.zeros(shape, dtype=np.float64)
    for ax, n in enumerate(shape):
        f = np.fft.fftfreq(n)
        bshape = [1] * d
        bshape[ax] = n
        k2 = k2 + float(beta[ax]) * (f.reshape(bshape) ** 2)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0.0, k2 ** (-(H + 0.5 * d) / 2.0), 0.0)
    field_ = np.real(np.fft.ifftn(spec * amp))
    sd = field_.std()
    if sd == 0.0:
        return np.zeros(shape)
    return (field_ - field_.mean()) / sd


def bonds_from_node_field(phi: np.ndarray, sigma: float, periodic: bool = False) -> List[np.ndarray]:
    """ln g of a bond = sigma * (mean of its two end-node field values).

    The field is periodic, so the last-plane entry of direction k joins the
    last and the first plane; it is kept for a periodic lattice, else zeroed.
    """
    dim = phi.ndim
    out = []
    for k in range(dim):
        ax = dim - 1 - k
        nb = np.roll(phi, -1, axis=ax)       # value at i + e_k, wrapped on the last plane
        out.append(np.exp(sigma * 0.5 * (phi + nb)))
    return out if periodic else clear_edge_bonds(out)


def iid_lognormal(dim: int, nx: int, ny: int, nz: int, sigma: float,
                  rng: np.random.Generator, mu: float = 0.0, periodic: bool = False) -> List[np.ndarray]:
    """ln g ~ N(mu, sigma^2) independently per bond (direction 0 first, then 1, then 2).

    Every entry is drawn; the last-plane entries are zeroed unless ``periodic``.
    """
    shape = node_shape(dim, nx, ny, nz)
    g = [np.exp(mu + sigma * rng.standard_normal(shape)) for _ in range(dim)]
    return [np.ascontiguousarray(a) for a in g] if periodic else clear_edge_bonds(g)


def dilute_iid(g: List[np.ndarray], occupancy: float, rng: np.random.Generator) -> List[np.ndarray]:
    """Keep each bond independently with probability ``occupancy`` (u < occupancy)."""
    out = []
    for a in g:
        u = rng.random(a.shape)
        out.append(np.where(u < occupancy, a, 0.0))
    return out


def dilute_rank(g: List[np.ndarray], q: float, wrap: Optional[Sequence[bool]] = None) -> List[np.ndarray]:
    """Remove the fraction ``q`` of lattice bonds with the smallest conductance.

    Correlated dilution of Sec. VI.B: sort all bonds by conductance and cut the
    lowest ``floor(q * n_bonds)``; ties are broken by bond order (direction,
    then node index) so the result is reproducible. ``wrap[k]`` counts the
    last-plane entries of direction k as bonds (periodic sides).
    """
    dim = len(g)
    shape = g[0].shape
    vals, keys = [], []
    for k, a in enumerate(g):
        valid = edge_valid(dim, shape, k).ravel()
        if wrap is not None and wrap[k]:
            valid = np.ones_like(valid)
        idx = np.nonzero(valid)[0]
        vals.append(a.ravel()[idx])
        keys.append(np.stack([np.full(idx.size, k), idx], axis=1))
    allv = np.concatenate(vals)
    allk = np.concatenate(keys)
    n_cut = int(math.floor(q * allv.size))
    order = np.lexsort((allk[:, 1], allk[:, 0], allv))
    cut = allk[order[:n_cut]]
    out = [a.copy() for a in g]
    for k in range(dim):
        sel = cut[cut[:, 0] == k, 1]
        out[k].ravel()[sel] = 0.0
    return out


# ----------------------------------------------------------------------------- workloads

def uniform_network(dim: int, nx: int, ny: int, nz: int = 1, g0: float = 1.0, axis: int = 0,
                    periodic: bool = False) -> Network:
    shape = node_shape(dim, nx, ny, nz)
    g = [np.full(shape, g0) for _ in range(dim)]
    if not periodic:
        g = clear_edge_bonds(g)
    return Network(dim, nx, ny, nz if dim == 3 else 1, g, axis, {"kind": "uniform", "g0": g0}, periodic)


def iid_network(dim: int, nx: int, ny: int, nz: int = 1, sigma: float = 1.0,
                occupancy: float = 1.0, index: int = 0, axis: int = 0, periodic: bool = False) -> Network:
    rng = rng_for(index)
    g = iid_lognormal(dim, nx, ny, nz, sigma, rng, periodic=periodic)
    if occupancy < 1.0:
        g = dilute_iid(g, occupancy, rng)
    return Network(dim, nx, ny, nz if dim == 3 else 1, g, axis,
                   {"kind": "iid", "sigma": sigma, "occupancy": occupancy, "index": index}, periodic)


def fbm_network(dim: int, nx: int, ny: int, nz: int = 1, H: float = 0.7, sigma: float = 1.0,
                occupancy: float = 1.0, index: int = 0, axis: int = 0,
                beta: Optional[Sequence[float]] = None, rank_q: Optional[float] = None,
                periodic: bool = False) -> Network:
    """FBM log-normal network: node field -> bond ln g -> optional dilution.

    With ``periodic`` the sides wrap around (Sec. II); rank dilution then
    counts the wrap bonds of the directions other than ``axis``.
    """
    rng = rng_for(index)
    shape = node_shape(dim, nx, ny, nz)
    phi = fbm_field(shape, H, rng, beta=beta)
    g = bonds_from_node_field(phi, sigma, periodic=periodic)
    if rank_q is not None:
        wrap = [periodic and k != axis for k in range(dim)]
        g = dilute_rank([a if wrap[k] else clear_edge(a, k) for k, a in enumerate(g)], rank_q, wrap)
    elif occupancy < 1.0:
        g = dilute_iid(g, occupancy, rng)
    return Network(dim, nx, ny, nz if dim == 3 else 1, g, axis,
                   {"kind": "fbm", "H": H, "sigma": sigma, "occupancy": occupancy,
                    "index": index, "beta": None if beta is None else list(beta), "rank_q": rank_q},
                   periodic)


def stratified_network(n: int, H: float = 0.8, sigma: float = 2.0, occupancy: float = 1.0,
                       index: int = 0, axis: int = 0, nx: Optional[int] = None,
                       ny: Optional[int] = None, nz: Optional[int] = None, periodic: bool = False) -> Network:
    """3D layered medium: ln g follows a 1D FBM profile phi(z) (H, standardised, times sigma).

    x- and y-bonds in layer z get ``sigma * phi[z]``; the z-bond from layer z to
    z+1 gets ``sigma * (phi[z] + phi[z+1]) / 2``. Dilution is i.i.d. per bond.
    """
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = rng_for(index)
    phi = fbm_field((nz,), H, rng)
    shape = (nz, ny, nx)
    lg_xy = (sigma * phi)[:, None, None] * np.ones(shape)
    phi_up = np.roll(phi, -1)                # the last layer's z-bond wraps to layer 0
    lg_z = (sigma * 0.5 * (phi + phi_up))[:, None, None] * np.ones(shape)
    g = [np.exp(lg_xy), np.exp(lg_xy), np.exp(lg_z)]
    if not periodic:
        g = clear_edge_bonds(g)
    if occupancy < 1.0:
        g = dilute_iid(g, occupancy, rng)
    return Network(3, nx, ny, nz, g, axis,
                   {"kind": "stratified", "H": H, "sigma": sigma, "occupancy": occupancy,
                    "index": index, "phi": phi}, periodic)


# Named workloads: the five cases the benchmark and the parity tests use.

def workload_iid_2d_128(index: int = 0) -> Network:
    """128 x 128 square lattice, ln g ~ N(0, 1) i.i.d., no dilution, flow along x."""
    return iid_network(2, 128, 128, 1, sigma=1.0, occupancy=1.0, index=index, axis=0)


def workload_fbm_2d_2048(index: int = 0, n: int = 2048) -> Network:
    """2048^2 square lattice, 2D FBM ln g (H=0.7, sigma=1.5), i.i.d. occupancy 0.6."""
    return fbm_network(2, n, n, 1, H=0.7, sigma=1.5, occupancy=0.6, index=index, axis=0)


def workload_strat_3d_256(index: int = 0, n: int = 256, occupancy: float = 0.27) -> Network:
    """256^3 simple-cubic lattice, layered 1D-FBM ln g along z (H=0.8, sigma=2), occupancy 0.27."""
    return stratified_network(n, H=0.8, sigma=2.0, occupancy=occupancy, index=index, axis=0)


@dataclass
class BatchSpec:
    dim: int
    side: int
    H: float
    occupancy: float
    index: int


def batch_specs(count: int = 512, seed_offset: int = 0,
                side2d: Tuple[int, int] = (64, 1024), side3d: Tuple[int, int] = (32, 128)) -> List[BatchSpec]:
    """Sizes and parameters of the mixed batch (half 2D, half 3D, interleaved)."""
    rng = rng_for(10_000_000 + seed_offset)
    out = []
    for i in range(count):
        dim = 2 if i % 2 == 0 else 3
        if dim == 2:
            side = int(rng.integers(side2d[0], side2d[1] + 1))
            occ = float(rng.uniform(0.55, 1.0))
        else:
            side = int(rng.integers(side3d[0], side3d[1] + 1))
            occ = float(rng.uniform(0.3, 1.0))
        H = float(rng.uniform(0.5, 0.9))
        out.append(BatchSpec(dim, side, H, occ, 20_000_000 + seed_offset + i))
    return out


def batch_network(spec: BatchSpec, sigma: float = 1.0) -> Network:
    s = spec.side
    if spec.dim == 2:
        return fbm_network(2, s, s, 1, H=spec.H, sigma=sigma, occupancy=spec.occupancy,
                           index=spec.index, axis=0)
    return fbm_network(3, s, s, s, H=spec.H, sigma=sigma, occupancy=spec.occupancy,
                       index=spec.index, axis=0)


@dataclass
class AnisoSpec:
    H: float
    ratio: float          # beta_x / beta_y of Eq. 2 (> 1: strata parallel to x)
    index: int


def aniso_specs(H_values: Sequence[float] = (0.75, 0.35), ratios: Sequence[float] = (1, 2, 4, 8, 16),
                seeds: int = 16, seed_offset: int = 0) -> List[AnisoSpec]:
    """The K_x / K_y study of Sec. VI.B (Fig. 10): for every Hurst exponent and
    anisotropy ratio, `seeds` independent networks (seed streams 30,000,000 +)."""
    out = []
    k = 0
    for H in H_values:
        for ratio in ratios:
            for _ in range(seeds):
                out.append(AnisoSpec(float(H), float(ratio), 30_000_000 + seed_offset + k))
                k += 1
    return out


def aniso_network(spec: AnisoSpec, n: int = 512, sigma: float = 1.5, rank_q: Optional[float] = None) -> Network:
    """2D n x n network with the anisotropic spectrum of Eq. 2: beta_y = 1 and
    beta_x = ratio (numpy axes are (y, x)), optionally rank-diluted (Sec. VI.B)."""
    net = fbm_network(2, n, n, 1, H=spec.H, sigma=sigma, index=spec.index, axis=0,
                      beta=[1.0, spec.ratio], rank_q=rank_q)
    net.meta["ratio"] = spec.ratio
    return net


@dataclass
class StreamRequest:
    t_arrival: float
    dim: int
    side: int
    occupancy: float
    index: int


def stream_requests(count: int, rate_per_s: float, n_min: float = 1e4, n_max: float = 3e7,
                    seed_offset: int = 0) -> List[StreamRequest]:
    """Poisson arrivals; node count log-uniform in [n_min, n_max]; 2D/3D 50/50."""
    rng = rng_for(30_000_000 + seed_offset)
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        dim = 2 if rng.random() < 0.5 else 3
        n = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
        side = max(3, int(round(n ** (1.0 / dim))))
        occ = float(rng.uniform(0.3, 1.0))
        out.append(StreamRequest(t, dim, side, occ, 40_000_000 + seed_offset + i))
    return out


def stream_network(req: StreamRequest, H: float = 0.75, sigma: float = 1.5) -> Network:
    s = req.side
    if req.dim == 2:
        return fbm_network(2, s, s, 1, H=H, sigma=sigma, occupancy=req.occupancy, index=req.index, axis=0)
    return fbm_network(3, s, s, s, H=H, sigma=sigma, occupancy=req.occupancy, index=req.index, axis=0)
