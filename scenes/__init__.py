"""Seeded synthetic inputs shared by the GPU path, the oracle tests and the bench.

This module holds no arithmetic of the sampling / rendering method. It only
draws the inputs the method consumes:

* an analytic radiance field (Gaussian density blobs, an optional opaque
  background shell, colour maps) standing in for a user's NeRF,
* occupancy-grid bits obtained from a conservative upper bound of that field
  (the grid estimator's state, supplied as an input),
* ray bundles (sphere-origin rays, pinhole cameras, multi-camera rigs),
* upstream gradients, proposal-MLP initial weights and jitter.

Seeds follow one convention: 0 blob centres, 1 colour maps, 2 cameras/rays,
3 upstream gradients, 4 MLP init, 5 jitter.  Every generator uses numpy's
PCG64 bit generator so that a (seed, shape) pair gives the same numbers on
every machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BLOBS, SEED_COLOUR, SEED_RAYS, SEED_GRADS, SEED_MLP, SEED_JITTER = 0, 1, 2, 3, 4, 5


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# analytic field
# ----------------------------------------------------------------------------
@dataclass
class BlobField:
    """sigma(x) = sum_b peak * exp(-|x-c_b|^2 / (2 w^2))  [+ shell term].

    rgb(x) = density-weighted mix of sigmoid(A x + b) (blobs) and
    sigmoid(A2 x/|x| + b2) (shell); with no shell it is sigmoid(A x + b).
    """
    centres: np.ndarray            # [B,3] float64
    peak: float = 50.0
    width: float = 0.1
    A: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))
    b: np.ndarray = field(default_factory=lambda: np.zeros(3))
    shell: bool = False
    shell_radius: float = 10.0
    shell_width: float = 0.5
    shell_peak: float = 20.0
    A2: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))
    b2: np.ndarray = field(default_factory=lambda: np.zeros(3))

    @property
    def n_blobs(self) -> int:
        return int(self.centres.shape[0])

    def packed_params(self) -> np.ndarray:
        """Flat float64 parameter vector (layout shared by both field kernels).

        [0] n_blobs, [1] peak, [2] width, [3] shell flag, [4] shell radius,
        [5] shell width, [6] shell peak, [7:16] A (row-major), [16:19] b,
        [19:28] A2, [28:31] b2, [32:32+3B] centres.
        """
        p = np.zeros(32 + 3 * self.n_blobs, dtype=np.float64)
        p[0] = self.n_blobs
        p[1], p[2] = self.peak, self.width
        p[3] = 1.0 if self.shell else 0.0
        p[4], p[5], p[6] = self.shell_radius, self.shell_width, self.shell_peak
        p[7:16] = np.asarray(self.A, np.float64).reshape(-1)
        p[16:19] = self.b
        p[19:28] = np.asarray(self.A2, np.float64).reshape(-1)
        p[28:31] = self.b2
        p[32:] = self.centres.reshape(-1)
        return p


def blob_field(n_blobs: int, *, shell: bool = False, peak: float = 50.0,
               width: float = 0.1, seed_blobs: int = SEED_BLOBS,
               seed_colour: int = SEED_COLOUR) -> BlobField:
    """Blob centres U[-1,1]^3 (seed 0), colour map A~U[-2,2], b~U[-.5,.5] (seed 1)."""
    c = rng(seed_blobs).uniform(-1.0, 1.0, size=(n_blobs, 3))
    g = rng(seed_colour)
    A = g.uniform(-2.0, 2.0, size=(3, 3))
    b = g.uniform(-0.5, 0.5, size=3)
    A2 = g.uniform(-2.0, 2.0, size=(3, 3))
    b2 = g.uniform(-0.5, 0.5, size=3)
    return BlobField(centres=c, peak=peak, width=width, A=A, b=b, shell=shell,
                     A2=A2, b2=b2)


# ----------------------------------------------------------------------------
# occupancy grids (conservative bound of the analytic field)
# ----------------------------------------------------------------------------
def _axis_gauss_bound(centres_1d: np.ndarray, lo: np.ndarray, hi: np.ndarray,
                      width: float) -> np.ndarray:
    """[B, res] max over each cell's 1-D extent of exp(-d^2/(2w^2))."""
    c = centres_1d[:, None]
    d = np.maximum(0.0, np.maximum(lo[None, :] - c, c - hi[None, :]))
    return np.exp(-d * d / (2.0 * width * width))


def occupancy_bits(fld: BlobField, res: int, center=(0.0, 0.0, 0.0),
                   half_extent: float = 1.5, tau: float = 0.01) -> np.ndarray:
    """Bit-packed grid (uint32 words, cell index x + res*(y + res*z), x fastest).

    Cell occupied iff an upper bound of sigma over the cell box exceeds tau:
    sum_b peak * prod_a exp(-dist_a^2/(2w^2)) (+ shell bound).  Returns
    uint32[res^3/32].
    """
    center = np.asarray(center, np.float64)
    edges = [center[a] - half_extent + (2.0 * half_extent) * np.arange(res + 1) / res
             for a in range(3)]
    gx, gy, gz = (_axis_gauss_bound(fld.centres[:, a], edges[a][:-1], edges[a][1:], fld.width)
                  for a in range(3))
    bound = fld.peak * np.einsum("bi,bj,bk->kji", gx, gy, gz, optimize=True)  # [z,y,x]
    if fld.shell:
        lo = [e[:-1] for e in edges]
        hi = [e[1:] for e in edges]
        # distance range from the origin to each cell box
        near = [np.maximum(0.0, np.maximum(lo[a], -hi[a])) for a in range(3)]
        far = [np.maximum(np.abs(lo[a]), np.abs(hi[a])) for a in range(3)]
        dmin = np.sqrt(near[2][:, None, None] ** 2 + near[1][None, :, None] ** 2
                       + near[0][None, None, :] ** 2)
        dmax = np.sqrt(far[2][:, None, None] ** 2 + far[1][None, :, None] ** 2
                       + far[0][None, None, :] ** 2)
        R = fld.shell_radius
        gap = np.where(R < dmin, dmin - R, np.where(R > dmax, R - dmax, 0.0))
        bound = bound + fld.shell_peak * np.exp(-gap * gap / (2.0 * fld.shell_width ** 2))
    occ = (bound > tau).reshape(-1)
    return pack_bits(occ)


def pack_bits(occ: np.ndarray) -> np.ndarray:
    """bool[res^3] (x fastest) -> uint32 words, bit i of word w = cell 32w+i."""
    occ = np.asarray(occ, dtype=bool).reshape(-1)
    assert occ.size % 32 == 0
    b = occ.reshape(-1, 32).astype(np.uint64)
    words = (b << np.arange(32, dtype=np.uint64)[None, :]).sum(axis=1)
    return words.astype(np.uint32)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    w = np.asarray(words, np.uint32).astype(np.uint64)
    bits = (w[:, None] >> np.arange(32, dtype=np.uint64)[None, :]) & 1
    return bits.reshape(-1)[:n].astype(bool)


def cascade_bits(fld: BlobField, res: int, n_levels: int, half_extent0: float = 1.5,
                 tau: float = 0.01) -> np.ndarray:
    """Concatenated grids for nested cubes of half-extent h0*2^l, l=0..L-1."""
    return np.concatenate([occupancy_bits(fld, res, half_extent=half_extent0 * 2 ** l, tau=tau)
                           for l in range(n_levels)])


def random_bits(res: int, p: float, seed: int) -> np.ndarray:
    """Uniformly random occupancy (for edge / property tests)."""
    return pack_bits(rng(seed).random(res ** 3) < p)


# ----------------------------------------------------------------------------
# rays
# ----------------------------------------------------------------------------
def _normalize(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def sphere_rays(n: int, radius: float = 3.0, target_half: float = 0.5,
                seed: int = SEED_RAYS):
    """Origins uniform on a sphere, directions towards U[-h,h]^3 targets.

    Returns float32 (o [n,3], d [n,3]); directions normalised in float64.
    """
    g = rng(seed)
    o = radius * _normalize(g.standard_normal((n, 3)))
    tgt = g.uniform(-target_half, target_half, size=(n, 3))
    d = _normalize(tgt - o)
    return o.astype(np.float32), d.astype(np.float32)


def look_at_camera(eye, width: int, height: int, fov_deg: float, *, fov_axis="y",
                   target=(0.0, 0.0, 0.0), up=(0.0, 0.0, 1.0)):
    """Pinhole rays through pixel centres; fov measured along fov_axis."""
    eye = np.asarray(eye, np.float64)
    fwd = _normalize(np.asarray(target, np.float64) - eye)
    right = np.cross(fwd, np.asarray(up, np.float64))
    if np.linalg.norm(right) < 1e-9:
        right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right = _normalize(right)
    upv = np.cross(right, fwd)
    span = width if fov_axis == "x" else height
    f = 0.5 * span / math.tan(0.5 * math.radians(fov_deg))
    j, i = np.meshgrid(np.arange(height, dtype=np.float64), np.arange(width, dtype=np.float64),
                       indexing="ij")
    px = (i + 0.5 - 0.5 * width) / f
    py = -(j + 0.5 - 0.5 * height) / f
    d = _normalize(fwd[None, None, :] + px[..., None] * right[None, None, :]
                   + py[..., None] * upv[None, None, :]).reshape(-1, 3)
    o = np.broadcast_to(eye, d.shape)
    return o.astype(np.float32).copy(), d.astype(np.float32)


def random_eyes(n: int, radius: float = 3.0, seed: int = SEED_RAYS) -> np.ndarray:
    return radius * _normalize(rng(seed).standard_normal((n, 3)))


def pinhole_rays(width: int = 1024, height: int = 1024, fov_deg: float = 40.0,
                 radius: float = 3.0, seed: int = SEED_RAYS):
    """One camera at a seeded point of the radius-r sphere looking at the origin."""
    eye = random_eyes(1, radius, seed)[0]
    return look_at_camera(eye, width, height, fov_deg)


def rig_rays(n_cams: int = 8, width: int = 512, height: int = 256, fov_deg: float = 60.0,
             radius: float = 3.0, seed: int = SEED_RAYS):
    """n_cams seeded cameras on the sphere, horizontal fov, concatenated rays."""
    eyes = random_eyes(n_cams, radius, seed)
    os, ds = zip(*(look_at_camera(e, width, height, fov_deg, fov_axis="x") for e in eyes))
    return np.concatenate(os), np.concatenate(ds)


def rig_camera(index: int, width: int = 512, height: int = 256, fov_deg: float = 60.0,
               radius: float = 3.0, seed: int = SEED_RAYS):
    """Camera `index` of the seeded rig's eye sequence.  The eyes are drawn in
    order from one generator, so cameras 0..n-1 are those of rig_rays(n) and
    cameras n, n+1, ... are further views of the same rig (held-out views)."""
    eye = random_eyes(index + 1, radius, seed)[index]
    return look_at_camera(eye, width, height, fov_deg, fov_axis="x")


# ----------------------------------------------------------------------------
# other seeded inputs
# ----------------------------------------------------------------------------
def upstream_grads(n: int, channels: int = 3, seed: int = SEED_GRADS) -> np.ndarray:
    return rng(seed).standard_normal((n, channels)).astype(np.float32)


def uniform_jitter(shape, seed: int = SEED_JITTER) -> np.ndarray:
    return rng(seed).random(shape).astype(np.float32)


def mlp_init(hidden: int, seed: int = SEED_MLP) -> np.ndarray:
    """Seeded He-uniform initial parameters of the proposal network.

    Layout W1 [H,39], b1 [H], W2 [H,H], b2 [H], w3 [H], b3 (float32); weight
    matrices ~ U(-sqrt(6/fan_in), sqrt(6/fan_in)), biases zero.
    """
    g = rng(seed)
    H = hidden
    W1 = g.uniform(-1, 1, (H, 39)) * np.sqrt(6.0 / 39)
    W2 = g.uniform(-1, 1, (H, H)) * np.sqrt(6.0 / H)
    w3 = g.uniform(-1, 1, H) * np.sqrt(6.0 / H)
    z = np.zeros
    return np.concatenate([W1.ravel(), z(H), W2.ravel(), z(H), w3, z(1)]).astype(np.float32)


# ----------------------------------------------------------------------------
# workload configurations
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    fld: BlobField
    bits: np.ndarray
    res: int
    n_levels: int
    half_extent0: float
    rays_o: np.ndarray
    rays_d: np.ndarray
    dt0: float
    t_min: float = 1e-4
    near: float = 0.0
    far: float = float("inf")
    grads: np.ndarray | None = None

    @property
    def n_rays(self) -> int:
        return int(self.rays_o.shape[0])


IMAGE_STEP = math.sqrt(3.0) * 3.0 / 1024.0


def tiny(n_rays: int = 4096) -> Workload:
    """8 blobs, 64^3 grid over [-1.5,1.5]^3, sphere rays, step 0.005."""
    f = blob_field(8)
    o, d = sphere_rays(n_rays)
    return Workload("tiny", f, occupancy_bits(f, 64), 64, 1, 1.5, o, d, 0.005,
                    grads=upstream_grads(n_rays))


def image(width: int = 1024, height: int = 1024) -> Workload:
    """32 blobs, 128^3 grid, 1024x1024 pinhole camera (fov 40), step sqrt(3)*3/1024."""
    f = blob_field(32)
    o, d = pinhole_rays(width, height)
    return Workload("image", f, occupancy_bits(f, 128), 128, 1, 1.5, o, d, IMAGE_STEP,
                    grads=upstream_grads(o.shape[0]))


def unbounded(width: int = 512, height: int = 256, n_cams: int = 8, n_levels: int = 4,
              res: int = 128) -> Workload:
    """64 blobs + background shell, 4 nested 128^3 grids, 8 cameras."""
    f = blob_field(64, shell=True)
    o, d = rig_rays(n_cams, width, height)
    return Workload("unbounded", f, cascade_bits(f, res, n_levels), res, n_levels, 1.5, o, d,
                    IMAGE_STEP, grads=upstream_grads(o.shape[0]))
