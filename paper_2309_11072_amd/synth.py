"""Seeded synthetic Radiance (RGBE) images.

This module only makes inputs: it holds none of the encoder's arithmetic and is
shared by the GPU tests, the oracle tests and the benchmark.  The public HDR
photo sets the paper measures on are not available, so these images stand in
for them with the shape the paper uses (full-colour Radiance pixels, Sec. IV)
and a controllable exponent spread.

Recipe (per image):
  1. Z ~ N(0, 1) of shape H x W from numpy's PCG64(seed);
  2. Z is smoothed by a Gaussian of `smooth` pixels (reflect borders) and
     standardised (empirical mean removed, divided by the empirical standard
     deviation; a field too small to vary is taken as flat);
  3. log2 luminance = sigma_l * Z;
  4. per-channel chroma ratios rho_c ~ U[0.5, 2] on a `cell`-pixel grid,
     bilinearly interpolated and normalised to unit Rec. 709 luminance;
  5. f_c = 2^(log2 luminance) * rho_c;
  6. optionally a Bernoulli(spec_frac) mask multiplies f by 2^spec_stops;
  7. packing into RGBE with the forward converter of Sec. II.A (Eq. 1-2),
     read through frexp so the largest mantissa stays in [128, 255]: with
     v = max_c f_c = m 2^e, m in [0.5, 1): E = e + 128, M_c = floor(f_c 2^(8-e)).
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass

import numpy as np
from scipy.ndimage import gaussian_filter


def pack_rgbe(f: np.ndarray) -> np.ndarray:
    """float64 [H, W, 3] (non-negative) -> uint8 [H, W, 4] (R, G, B, E)."""
    f = np.asarray(f, np.float64)
    v = f.max(axis=-1)
    m, e = np.frexp(v)
    lit = v >= 2.0 ** -128
    E = np.where(lit, e + 128, 0)
    if np.any(E > 255):
        raise ValueError("value too large for RGBE")
    M = np.floor(np.ldexp(f, (8 - e)[..., None]))
    M = np.where(lit[..., None], M, 0)
    out = np.empty(f.shape[:2] + (4,), np.uint8)
    out[..., :3] = M.astype(np.uint8)
    out[..., 3] = E.astype(np.uint8)
    return out


def _bilinear(grid: np.ndarray, H: int, W: int, cell: int) -> np.ndarray:
    gy = (np.arange(H) + 0.5) / cell
    gx = (np.arange(W) + 0.5) / cell
    y0 = np.floor(gy).astype(np.int64)
    x0 = np.floor(gx).astype(np.int64)
    wy = (gy - y0)[:, None]
    wx = (gx - x0)[None, :]
    g = grid
    a = g[:, y0][:, :, x0]
    b = g[:, y0][:, :, x0 + 1]
    c = g[:, y0 + 1][:, :, x0]
    d = g[:, y0 + 1][:, :, x0 + 1]
    return (a * (1 - wx) + b * wx) * (1 - wy) + (c * (1 - wx) + d * wx) * wy


def generate(H: int, W: int, sigma_l: float, seed: int, spec_frac: float = 0.0,
             spec_stops: float = 10.0, smooth: float = 8.0, cell: int = 32) -> np.ndarray:
    """One seeded synthetic RGBE image, uint8 [H, W, 4]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((H, W))
    z = gaussian_filter(z, smooth, mode="reflect")
    z -= z.mean()
    sd = z.std()
    z = z / sd if sd > 1e-6 else np.zeros_like(z)
    log2l = sigma_l * z
    gh, gw = H // cell + 2, W // cell + 2
    rho = _bilinear(rng.uniform(0.5, 2.0, (3, gh, gw)), H, W, cell)
    rho /= (0.2126 * rho[0] + 0.7152 * rho[1] + 0.0722 * rho[2])[None]
    f = np.exp2(log2l)[..., None] * np.moveaxis(rho, 0, -1)
    if spec_frac > 0:
        mask = rng.random((H, W)) < spec_frac
        f[mask] *= 2.0 ** spec_stops
    return pack_rgbe(f)


def generate_torch(H: int, W: int, sigma_l: float, seed: int, spec_frac: float = 0.0, spec_stops: float = 10.0,
                   smooth: float = 8.0, cell: int = 32, device="cuda"):
    """The same recipe drawn with torch's seeded generator on `device` (for
    benchmark batches of hundreds of megapixels, where the numpy generator
    would take minutes).  The random streams differ from generate(); the
    distributions, the smoothing (Gaussian truncated at 4 sigma, reflected
    borders where the image is large enough, replicated otherwise), the chroma
    grid and the RGBE packing are the same.  Returns uint8 [H, W, 4] on
    `device`."""
    import torch
    import torch.nn.functional as F
    g = torch.Generator(device=device).manual_seed(int(seed))
    z = torch.randn((1, 1, H, W), generator=g, device=device, dtype=torch.float32)
    r = int(4 * smooth + 0.5)
    k = [math.exp(-0.5 * (i / smooth) ** 2) for i in range(-r, r + 1)]
    k = [v / sum(k) for v in k]
    mode_x = "reflect" if W > r else "replicate"
    mode_y = "reflect" if H > r else "replicate"
    # Separable convolution as a sum of shifted copies (plain elementwise
    # work, no convolution library).
    zp = F.pad(z, (r, r, 0, 0), mode=mode_x)[0, 0]
    acc = torch.zeros((H, W), device=device, dtype=torch.float32)
    for i, v in enumerate(k):
        acc += v * zp[:, i:i + W]
    zp = F.pad(acc[None, None], (0, 0, r, r), mode=mode_y)[0, 0]
    acc = torch.zeros((H, W), device=device, dtype=torch.float32)
    for i, v in enumerate(k):
        acc += v * zp[i:i + H, :]
    z = acc.double()
    del zp, acc
    z = z - z.mean()
    sd = float(z.std(unbiased=False))
    z = z / sd if sd > 1e-6 else torch.zeros_like(z)
    log2l = sigma_l * z
    gh, gw = H // cell + 2, W // cell + 2
    grid = 0.5 + 1.5 * torch.rand((3, gh, gw), generator=g, device=device, dtype=torch.float64)
    gy = (torch.arange(H, device=device, dtype=torch.float64) + 0.5) / cell
    gx = (torch.arange(W, device=device, dtype=torch.float64) + 0.5) / cell
    y0, x0 = gy.floor().long(), gx.floor().long()
    wy, wx = (gy - y0)[:, None], (gx - x0)[None, :]
    rho = torch.empty((3, H, W), device=device, dtype=torch.float64)
    for c in range(3):
        a = grid[c][y0][:, x0]
        b = grid[c][y0][:, x0 + 1]
        cc = grid[c][y0 + 1][:, x0]
        d = grid[c][y0 + 1][:, x0 + 1]
        rho[c] = (a * (1 - wx) + b * wx) * (1 - wy) + (cc * (1 - wx) + d * wx) * wy
    rho /= (0.2126 * rho[0] + 0.7152 * rho[1] + 0.0722 * rho[2])[None]
    f = torch.exp2(log2l)[None] * rho
    del rho, z, log2l
    if spec_frac > 0:
        mask = torch.rand((H, W), generator=g, device=device) < spec_frac
        f = torch.where(mask[None], f * 2.0 ** spec_stops, f)
    v = f.amax(dim=0)
    _, e = torch.frexp(v)
    lit = v >= 2.0 ** -128
    E = torch.where(lit, e + 128, torch.zeros_like(e))
    if bool((E > 255).any()):
        raise ValueError("value too large for RGBE")
    M = torch.floor(torch.ldexp(f, (8 - e)[None].double()))
    M = torch.where(lit[None], M, torch.zeros_like(M))
    out = torch.empty((H, W, 4), device=device, dtype=torch.uint8)
    out[..., :3] = M.permute(1, 2, 0).to(torch.uint8)
    out[..., 3] = E.to(torch.uint8)
    return out


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@dataclass
class ImageSpec:
    H: int
    W: int
    sigma_l: float
    q: int
    seed: int
    spec_frac: float = 0.0

    def make(self) -> np.ndarray:
        return generate(self.H, self.W, self.sigma_l, self.seed, self.spec_frac)

    def make_torch(self, device="cuda"):
        return generate_torch(self.H, self.W, self.sigma_l, self.seed, self.spec_frac, device=device)


ASPECTS = (4 / 3, 16 / 9, 1.0)


def _draw_sizes(n, a_lo, a_hi, rng):
    out = []
    for _ in range(n):
        A = rng.uniform(a_lo, a_hi)
        r = ASPECTS[rng.integers(0, 3)]
        W = int(round(np.sqrt(A * r)))
        H = int(round(A / W))
        out.append((max(H, 1), max(W, 1)))
    return out


def small_512x384() -> ImageSpec:
    """512x384 image, sigma 2.5, no speculars, q 90 (oracle-sized case)."""
    return ImageSpec(384, 512, 2.5, 90, 1)


def image_3840x2160() -> ImageSpec:
    """3840x2160 image, sigma 4, 5% speculars at +10 stops, q 75."""
    return ImageSpec(2160, 3840, 4.0, 75, 2, 0.05)


def batch_64_uneven(n: int = 64) -> list:
    """64 uneven images, 640x480 .. 3840x2160 pixels' worth of area,
    sigma in [1.5, 4], q in [50, 95]."""
    rng = np.random.Generator(np.random.PCG64(3))
    sizes = _draw_sizes(n, 640 * 480, 3840 * 2160, rng)
    return [ImageSpec(H, W, float(rng.uniform(1.5, 4.0)), int(rng.integers(50, 96)), 3000 + i)
            for i, (H, W) in enumerate(sizes)]


def learned_train_set() -> list:
    """Two 3840x2160 images (sigma 4, 5% speculars, q 75) to train the learned
    estimator on."""
    return [ImageSpec(2160, 3840, 4.0, 75, 4000 + i, 0.05) for i in range(2)]


def learned_train_set_wide(n: int = 8) -> list:
    """Training images over the parameter ranges of the batch workloads:
    eight 1920x1080 images, sigma in [1, 5], q in [30, 98], every second one
    with 5% speculars (the batch of 256 images has none, the 3840x2160
    workload has them)."""
    rng = np.random.Generator(np.random.PCG64(4010))
    return [ImageSpec(1080, 1920, float(rng.uniform(1.0, 5.0)), int(rng.integers(30, 99)), 4010 + i,
                      0.05 if i % 2 else 0.0) for i in range(n)]


def learned_eval_set() -> list:
    """Sixteen held-out 1920x1080 images with the same parameters."""
    return [ImageSpec(1080, 1920, 4.0, 75, 4100 + i, 0.05) for i in range(16)]


def batch_256_large(n: int = 256) -> list:
    """256 uneven images of 1 MP .. 33 MP, sigma in [1, 5], q in [30, 98]."""
    rng = np.random.Generator(np.random.PCG64(5))
    sizes = _draw_sizes(n, 1.0e6, 7680 * 4320, rng)
    return [ImageSpec(H, W, float(rng.uniform(1.0, 5.0)), int(rng.integers(30, 99)), 5000 + i)
            for i, (H, W) in enumerate(sizes)]


def random_model(seed: int, scale: int = 8, rq: str = "general") -> bytes:
    """A seeded random int8 estimator model (test input), within the value
    limits of the model format, with activations that neither vanish nor
    saturate on synthetic images.  rq chooses the library's requantisation
    path the model takes: "general" (multipliers above 1), "pow2" (every
    hidden multiplier 1, shifts differing within neuron pairs) or "pair"
    (multipliers 1, equal shifts in each pair (2k, 2k + 1), one pair per
    layer at the largest shift of that path, 22).  pow2 and pair models also
    have neurons whose biases push them past both ends of [0, 255]."""
    from . import model_format
    assert rq in ("general", "pow2", "pair")
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {
        "W1": np.zeros((32, 32), np.int8), "B1": rng.integers(-3000, 3000, (32, 32)),
        "m1": rng.integers(256, 1024, 32), "r1": rng.integers(14, 17, 32),
        "W2": rng.integers(-scale, scale + 1, (32, 32)), "B2": rng.integers(-2000, 4000, 32),
        "m2": rng.integers(256, 1024, 32), "r2": rng.integers(12, 15, 32),
        "W3": np.zeros((16, 32), np.int8), "B3": np.zeros(16, np.int64),
        "m3": np.full(16, 512), "r3": np.full(16, 6),
    }
    p["W1"][:, :27] = rng.integers(-scale, scale + 1, (32, 27))
    p["W3"][:3] = rng.integers(-scale, scale + 1, (3, 32))
    p["B3"][:3] = rng.integers(0, 2000, 3)
    if rq != "general":
        p["m1"] = np.ones(32, np.int64)
        p["r1"] = rng.integers(5, 10, 32)
        p["m2"] = np.ones(32, np.int64)
        p["r2"] = rng.integers(4, 10, 32)
        if rq == "pair":
            p["r1"][1::2] = p["r1"][0::2]
            p["r2"][1::2] = p["r2"][0::2]
            p["r1"][30:32] = 22
            p["r2"][30:32] = 22
        else:
            p["r1"][1::2] = np.where(p["r1"][1::2] == p["r1"][0::2], p["r1"][0::2] + 1, p["r1"][1::2])
        # neurons 0-1 of each hidden layer saturate at 255, 2-3 at 0
        p["B1"][:, 0:2] = rng.integers(150000, 260000, (32, 2))
        p["B1"][:, 2:4] = -rng.integers(150000, 260000, (32, 2))
        p["B2"][0:2] = rng.integers(150000, 260000, 2)
        p["B2"][2:4] = -rng.integers(150000, 260000, 2)
    return model_format.pack(p)
