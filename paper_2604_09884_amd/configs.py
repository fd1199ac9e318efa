"""Workload configurations for the INR-CT gradient step.

Each configuration fixes a scan geometry, a grid, a synthetic phantom recipe,
an INR architecture and the optimiser settings.  The paper (Sec. IV) runs a
2D fan-beam FORBILD study and a 3D cone-beam walnut study; neither data set
is available here, so these configurations describe seeded synthetic
stand-ins with the same structure (sparse views, FOV-masked grids, FFN and
SIREN INRs, minibatch subsampling as in Eq. (2)).

Conventions shared by every consumer (kernels, oracle, input generators):
  * the grid covers [-1, 1]^d with N points per axis, pitch h = 2/N, and
    centres c(i) = -1 + (i + 1/2) h; arrays are stored x fastest
    (2D: [y][x], 3D: [z][y][x]);
  * the FOV is the inscribed disc (2D) or the cylinder x^2 + y^2 <= 1 over
    all z (3D); n is the number of grid points inside it;
  * 2D parallel beam: view j has angle theta_j = j*span/V, ray direction
    (-sin, cos), detector axis (cos, sin), bin k at offset
    (k - (K-1)/2) * du;
  * 3D circular cone beam: view j has angle phi_j = j*span/V, source
    D_so (cos, sin, 0), detector centre -D_od (cos, sin, 0), detector axes
    e_u = (-sin, cos, 0) and e_v = (0, 0, 1), pixel (a, b) centred at
    ((a - (Nu-1)/2) du, (b - (Nv-1)/2) dv).
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass


@dataclass(frozen=True)
class INRArch:
    kind: str            # "ffn" (Fourier features + ReLU MLP), "siren" or "hash"
    in_dim: int          # d = 2 or 3
    n_freq: int          # Fourier frequencies F (encoding width 2F); 0 for SIREN
    sigma: float         # std of the Gaussian Fourier matrix B
    width: int           # hidden width W
    depth: int           # number of hidden layers L
    omega0: float = 30.0 # SIREN frequency factor
    # multi-resolution hash encoding (kind "hash"): levels, features per
    # level, log2 of the entries per level's table, coarsest and finest
    # resolution
    hash_levels: int = 16
    hash_feats: int = 2
    hash_log2_size: int = 19
    hash_base_res: int = 16
    hash_max_res: int = 512

    @property
    def enc_dim(self) -> int:
        if self.kind == "ffn":
            return 2 * self.n_freq
        if self.kind == "hash":
            return self.hash_levels * self.hash_feats
        return self.in_dim

    @property
    def n_table(self) -> int:
        """Trained hash-table entries (floats) ahead of the MLP."""
        if self.kind != "hash":
            return 0
        return self.hash_levels * (1 << self.hash_log2_size) * self.hash_feats

    def layer_dims(self):
        """(fan_in, fan_out) of each affine layer, output layer last."""
        dims = [(self.enc_dim, self.width)]
        dims += [(self.width, self.width)] * (self.depth - 1)
        dims.append((self.width, 1))
        return dims

    @property
    def n_params(self) -> int:
        return self.n_table + sum(i * o + o for i, o in self.layer_dims())

    def flops_forward(self) -> int:
        """Multiply-add FLOPs of one point's forward pass through the MLP."""
        return sum(2 * i * o for i, o in self.layer_dims())

    def flops_vjp(self) -> int:
        """FLOPs of one sample's forward + backward (weight grads and
        input grads for every layer past the first)."""
        dims = self.layer_dims()
        fwd = self.flops_forward()
        dw = sum(2 * i * o for i, o in dims)
        dx = sum(2 * i * o for i, o in dims[1:])
        return fwd + dw + dx


@dataclass(frozen=True)
class Problem:
    name: str
    dim: int
    N: int
    geometry: str               # "par2d", "fan2d" or "cone3d"
    n_views: int
    view_span: float            # radians covered by the views (endpoint excluded)
    n_u: int
    n_v: int                    # 1 in 2D
    du: float
    dv: float
    dso: float = 0.0            # source-to-isocentre (fan, cone)
    dod: float = 0.0            # isocentre-to-detector (fan, cone)
    n_ellipses: int = 10
    photons: float = 0.0        # 0 = noiseless
    arch: INRArch = None
    k_frac: float = 1.0         # |I| / n ; used when k_abs is 0
    k_abs: int = 0
    lr: float = 1e-3
    steps: int = 20
    mlp_dtype: str = "fp32"     # "fp32" or "bf16"
    chunk_points: int = 1 << 20
    seed_phantom: int = 1000
    seed_noise: int = 2000
    seed_init: int = 3000
    seed_sampler: int = 4000

    @property
    def h(self) -> float:
        return 2.0 / self.N

    @property
    def n_grid(self) -> int:
        return self.N ** self.dim

    @property
    def n_rays(self) -> int:
        return self.n_views * self.n_u * self.n_v

    def n_fov(self) -> int:
        N = self.N
        # integer form of c(ix)^2 + c(iy)^2 <= 1: (2ix+1-N)^2 + (2iy+1-N)^2 <= N^2
        cnt = 0
        for iy in range(N):
            a = 2 * iy + 1 - N
            rem = N * N - a * a
            if rem < 0:
                continue
            # number of ix with (2ix+1-N)^2 <= rem
            cnt += sum(1 for ix in range(N) if (2 * ix + 1 - N) ** 2 <= rem)
        return cnt * (N if self.dim == 3 else 1)

    def k(self, n: int | None = None) -> int:
        if self.k_abs:
            return self.k_abs
        n = self.n_fov() if n is None else n
        return max(1, int(round(self.k_frac * n)))

    def with_(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _ffn(d, F, W, L, sigma=10.0):
    return INRArch("ffn", d, F, sigma, W, L)


def _siren(d, W, L, omega0=30.0):
    return INRArch("siren", d, 0, 0.0, W, L, omega0)


# 2D parallel beam, 128^2, 60 views over 180 deg, 185 bins at the pixel pitch,
# 10 random ellipses, noiseless; FFN 2 -> 128 Fourier features (64
# frequencies, sigma 10) + 3 x 128 ReLU + linear; full sampling; 20 Adam
# steps at lr 1e-3; FP32.
C1 = Problem(
    name="par2d-128-ffn", dim=2, N=128, geometry="par2d", n_views=60,
    view_span=math.pi, n_u=185, n_v=1, du=2.0 / 128, dv=2.0 / 128,
    n_ellipses=10, photons=0.0, arch=_ffn(2, 64, 128, 3), k_frac=1.0,
    lr=1e-3, steps=20, mlp_dtype="fp32",
    seed_phantom=1001, seed_noise=2001, seed_init=3001, seed_sampler=4001)

# 2D parallel beam, 512^2, 90 views, 725 bins, Poisson noise at 1e5 photons;
# SIREN 2 -> 5 x 256 (omega0 30) -> 1; |I| = n/16; 2000 steps.
C2 = Problem(
    name="par2d-512-siren", dim=2, N=512, geometry="par2d", n_views=90,
    view_span=math.pi, n_u=725, n_v=1, du=2.0 / 512, dv=2.0 / 512,
    n_ellipses=10, photons=1e5, arch=_siren(2, 256, 5), k_frac=1.0 / 16,
    lr=1e-4, steps=2000, mlp_dtype="bf16",
    seed_phantom=1002, seed_noise=2002, seed_init=3002, seed_sampler=4002)

# Cone-beam world geometry shared by the 3D workloads: the volume spans
# [-1, 1]^3; source-isocentre 1000 and isocentre-detector 500 in units of
# four voxel pitches of a 256^3 grid (1/32), i.e. 31.25 and 15.625; a square
# detector 3.1 units wide.
CONE_DSO = 1000.0 / 32.0
CONE_DOD = 500.0 / 32.0
CONE_DET_WIDTH = 3.1

# 3D cone beam, 256^3, 60 views over 360 deg, 512^2 detector, 20 ellipsoids,
# noiseless; FFN 3 -> 512 Fourier features + 4 x 256 ReLU -> 1; 2^18 samples.
C3 = Problem(
    name="cone3d-256-ffn", dim=3, N=256, geometry="cone3d", n_views=60,
    view_span=2 * math.pi, n_u=512, n_v=512, du=CONE_DET_WIDTH / 512,
    dv=CONE_DET_WIDTH / 512, dso=CONE_DSO, dod=CONE_DOD, n_ellipses=20,
    photons=0.0, arch=_ffn(3, 256, 256, 4), k_abs=1 << 18, lr=1e-3,
    steps=1000, mlp_dtype="bf16",
    seed_phantom=1003, seed_noise=2003, seed_init=3003, seed_sampler=4003)

# 3D sparse-view cone beam, 501^3, 20 views over 360 deg, 768^2 detector,
# Poisson noise at 1e5 photons; FFN 3 -> 512 Fourier + 5 x 256 ReLU -> 1;
# |I| = 1% of n; grid evaluation in 2^20-point chunks.
C4 = Problem(
    name="cone3d-501-ffn", dim=3, N=501, geometry="cone3d", n_views=20,
    view_span=2 * math.pi, n_u=768, n_v=768, du=CONE_DET_WIDTH / 768,
    dv=CONE_DET_WIDTH / 768, dso=CONE_DSO, dod=CONE_DOD, n_ellipses=20,
    photons=1e5, arch=_ffn(3, 256, 256, 5), k_frac=0.01, lr=1e-3,
    steps=1000, mlp_dtype="bf16", chunk_points=1 << 20,
    seed_phantom=1004, seed_noise=2004, seed_init=3004, seed_sampler=4004)

# 2D fan beam, the acquisition of Sec. IV-A: 512^2, 180 views over 360 deg,
# 512 bins over the cone world geometry's 3.1-unit detector at its source
# and detector distances; 10 random ellipses (standing in for the FORBILD
# phantom), Poisson noise at 1e5 photons; FFN 2 -> 512 Fourier features +
# 4 x 256 ReLU -> 1 in BF16; |I| = n/16 (the paper's 2D minibatch).
C6 = Problem(
    name="fan2d-512-ffn", dim=2, N=512, geometry="fan2d", n_views=180,
    view_span=2 * math.pi, n_u=512, n_v=1, du=CONE_DET_WIDTH / 512,
    dv=CONE_DET_WIDTH / 512, dso=CONE_DSO, dod=CONE_DOD, n_ellipses=10,
    photons=1e5, arch=_ffn(2, 256, 256, 4), k_frac=1.0 / 16, lr=1e-3,
    steps=5000, mlp_dtype="bf16",
    seed_phantom=1006, seed_noise=2006, seed_init=3006, seed_sampler=4006)

# C6's fan-beam acquisition with the hash-encoding INR (the third
# architecture of Sec. IV): 16 levels of 2^19 two-feature entries from
# resolution 16 to 512, then 2 x 64 ReLU -> 1, FP32; |I| = n/16.
C7 = C6.with_(name="fan2d-512-hash",
              arch=INRArch("hash", 2, 0, 0.0, 64, 2, hash_levels=16, hash_feats=2,
                           hash_log2_size=19, hash_base_res=16, hash_max_res=512),
              mlp_dtype="fp32", seed_phantom=1007, seed_noise=2007, seed_init=3007,
              seed_sampler=4007)

CONFIGS = {"c1": C1, "c2": C2, "c3": C3, "c4": C4, "c6": C6, "c7": C7}


# C5, the serving mix: request kinds uniform over {2D-256, 2D-512, 3D-128,
# 3D-256}; 2D parallel beam with 60 or 90 views over 180 deg and ceil(N
# sqrt 2) bins rounded up to odd; 3D cone beam with 20, 40 or 60 views over
# 360 deg and a 2N x 2N detector on the shared world geometry; architecture
# uniform over {C1's FFN (full sampling, lr 1e-3), C2's SIREN (n/16, lr
# 1e-4)} with the request's input dimension; arrivals drawn from seed 5005.
def serving_mix(n_requests: int, seed: int = 5005, steps: int = 4):
    import numpy as np
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_requests):
        kind = ("2d-256", "2d-512", "3d-128", "3d-256")[rng.integers(4)]
        ffn = bool(rng.integers(2))
        N = int(kind.split("-")[1])
        dim = 2 if kind.startswith("2d") else 3
        if ffn:
            arch = _ffn(dim, 64, 128, 3)
            extra = dict(k_frac=1.0, lr=1e-3, mlp_dtype="fp32")
        else:
            arch = _siren(dim, 256, 5)
            extra = dict(k_frac=1.0 / 16, lr=1e-4, mlp_dtype="bf16")
        seeds = dict(seed_phantom=6000 + i, seed_noise=7000 + i, seed_init=8000 + i,
                     seed_sampler=9000 + i, steps=steps, n_ellipses=10, photons=0.0)
        if dim == 2:
            views = int((60, 90)[rng.integers(2)])
            bins = int(math.ceil(N * math.sqrt(2)))
            bins += 1 - bins % 2
            p = par2d_problem(N, views, bins, arch=arch, name=f"mix{i}-{kind}-{views}v",
                              **extra, **seeds)
        else:
            views = int((20, 40, 60)[rng.integers(3)])
            p = cone_problem(N, views, 2 * N, arch=arch, name=f"mix{i}-{kind}-{views}v",
                             n_ellipses=20, **{k: v for k, v in extra.items()},
                             **{k: v for k, v in seeds.items() if k != "n_ellipses"})
        out.append(p)
    return out


def cone_problem(N: int, n_views: int, det: int, **kw) -> Problem:
    """A cone-beam problem on the shared world geometry (detector det x det)."""
    base = dict(name=f"cone3d-{N}", dim=3, N=N, geometry="cone3d",
                n_views=n_views, view_span=2 * math.pi, n_u=det, n_v=det,
                du=CONE_DET_WIDTH / det, dv=CONE_DET_WIDTH / det,
                dso=CONE_DSO, dod=CONE_DOD)
    base.update(kw)
    return Problem(**base)


def fan2d_problem(N: int, n_views: int, n_bins: int, **kw) -> Problem:
    """A fan-beam problem on the cone world geometry's plane z = 0 (views
    over 360 deg, n_bins over the 3.1-unit detector)."""
    base = dict(name=f"fan2d-{N}", dim=2, N=N, geometry="fan2d",
                n_views=n_views, view_span=2 * math.pi, n_u=n_bins, n_v=1,
                du=CONE_DET_WIDTH / n_bins, dv=CONE_DET_WIDTH / n_bins,
                dso=CONE_DSO, dod=CONE_DOD)
    base.update(kw)
    return Problem(**base)


def par2d_problem(N: int, n_views: int, n_bins: int, **kw) -> Problem:
    base = dict(name=f"par2d-{N}", dim=2, N=N, geometry="par2d",
                n_views=n_views, view_span=math.pi, n_u=n_bins, n_v=1,
                du=2.0 / N, dv=2.0 / N)
    base.update(kw)
    return Problem(**base)
