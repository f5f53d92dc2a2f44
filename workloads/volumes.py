"""Procedural volumes (torch, CPU or GPU, float32 output).

Gradient noise is a project-written lattice noise in the manner of Perlin's
"Improving Noise" (2002): a gradient chosen by an integer hash of each lattice
corner among the twelve cube-edge directions, blended with the quintic fade
6t^5 - 15t^4 + 10t^3.  No third-party permutation table is used.  fBm sums
octaves with lacunarity 2 and gain 0.5, normalised by the sum of the gains so
that it stays within [-1, 1].
"""
import math

import torch

_GRADS = torch.tensor([[1, 1, 0], [-1, 1, 0], [1, -1, 0], [-1, -1, 0],
                       [1, 0, 1], [-1, 0, 1], [1, 0, -1], [-1, 0, -1],
                       [0, 1, 1], [0, -1, 1], [0, 1, -1], [0, -1, -1]], dtype=torch.float32)


def _hash3(i, j, k, seed):
    """32-bit integer hash of lattice coordinates (int64 tensors)."""
    m = 0xFFFFFFFF
    h = (i * 0x8DA6B343 + j * 0xD8163841 + k * 0xCB1AB31F + seed * 0x165667B1) & m
    h = ((h ^ (h >> 15)) * 0x2C1B3C6D) & m
    h = ((h ^ (h >> 12)) * 0x297A2D39) & m
    return h ^ (h >> 15)


def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def gradient_noise(p, seed=0):
    """Lattice gradient noise at points p (..., 3) float32; result roughly in [-1, 1]."""
    g = _GRADS.to(p.device)
    pf = torch.floor(p)
    f = p - pf
    pi = pf.to(torch.int64)
    u = _fade(f)
    out = torch.zeros(p.shape[:-1], dtype=p.dtype, device=p.device)
    for c in range(8):
        o = [(c >> 2) & 1, (c >> 1) & 1, c & 1]
        h = _hash3(pi[..., 0] + o[0], pi[..., 1] + o[1], pi[..., 2] + o[2], seed)
        gv = g[(h % 12)]
        d = f - torch.tensor(o, dtype=p.dtype, device=p.device)
        dot = (gv * d).sum(-1)
        w = torch.ones_like(out)
        for a in range(3):
            w = w * (u[..., a] if o[a] else 1.0 - u[..., a])
        out = out + w * dot
    return out


def fbm(p, octaves, seed=0, lacunarity=2.0, gain=0.5):
    total = torch.zeros(p.shape[:-1], dtype=p.dtype, device=p.device)
    amp, freq, norm = 1.0, 1.0, 0.0
    for o in range(octaves):
        total = total + amp * gradient_noise(p * freq, seed + 101 * o)
        norm += amp
        amp *= gain
        freq *= lacunarity
    return total / norm


def _grid(dims, device, origin=(0, 0, 0)):
    ax = [torch.arange(n, dtype=torch.float32, device=device) + o for n, o in zip(dims, origin)]
    return torch.meshgrid(*ax, indexing="ij")


def sphere_sdf(n=64, center=(32.0, 32.0, 32.0), radius=24.0, device="cpu"):
    """Signed distance to a sphere on an n^3 lattice, in voxel units (x-major grid)."""
    x, y, z = _grid((n, n, n), device)
    c = torch.tensor(center, dtype=torch.float64)
    d = torch.sqrt((x.double() - c[0]) ** 2 + (y.double() - c[1]) ** 2 + (z.double() - c[2]) ** 2)
    return (d - radius).to(torch.float32)


def two_spheres_sdf(n=128, centers=((50.0, 50.0, 50.0), (104.0, 24.0, 26.0)), radii=(24.0, 12.0),
                    device="cpu"):
    """Union of two disjoint spheres (signed distance, voxel units, n^3 lattice):
    a scene of separate clusters.  The surface of the first sphere passes
    through the corner shared by eight 64^3 blocks of the lattice."""
    x, y, z = _grid((n, n, n), device)
    out = None
    for c, r in zip(centers, radii):
        d = torch.sqrt((x.double() - c[0]) ** 2 + (y.double() - c[1]) ** 2 + (z.double() - c[2]) ** 2) - r
        out = d if out is None else torch.minimum(out, d)
    return out.to(torch.float32)


def noise_sphere_sdf(n=512, center=(256.0, 256.0, 256.0), radius=200.0, amplitude=20.0,
                     octaves=4, scale=64.0, seed=0, device="cpu", chunk=32):
    """Sphere displaced by fBm gradient noise: phi = |p - c| - R - amplitude * fbm(p / scale).

    Computed slab by slab along x to bound temporary memory."""
    out = torch.empty((n, n, n), dtype=torch.float32, device=device)
    for x0 in range(0, n, chunk):
        nx = min(chunk, n - x0)
        x, y, z = _grid((nx, n, n), device, (x0, 0, 0))
        p = torch.stack([x, y, z], -1)
        d = torch.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
        out[x0:x0 + nx] = d - radius - amplitude * fbm(p / scale, octaves, seed)
    return out


def fbm_cloud(n=1024, octaves=6, scale=256.0, seed=7, device="cpu", chunk=16):
    """Density 1/2 + 1/2 fbm(p / scale), clamped to [0, 1] (fog volume)."""
    out = torch.empty((n, n, n), dtype=torch.float32, device=device)
    for x0 in range(0, n, chunk):
        nx = min(chunk, n - x0)
        x, y, z = _grid((nx, n, n), device, (x0, 0, 0))
        p = torch.stack([x, y, z], -1)
        out[x0:x0 + nx] = (0.5 + 0.5 * fbm(p / scale, octaves, seed)).clamp(0.0, 1.0)
    return out


def saturated_fog(n=64, center=(32.0, 32.0, 32.0), radius=24.0, gain=3.0, amplitude=0.3, scale=16.0, seed=5,
                  device="cpu", chunk=32, levels=0):
    """Density clamp(gain (1 - |p - c| / R) + amplitude fbm(p / scale), 0, 1) on an n^3
    lattice (fog volume): a noisy ball whose core saturates at exactly 1, so the
    leaves inside the core are constant.  levels > 0 rounds the density down to a
    multiple of 1 / levels (terraces of constant density)."""
    out = torch.empty((n, n, n), dtype=torch.float32, device=device)
    for x0 in range(0, n, chunk):
        nx = min(chunk, n - x0)
        x, y, z = _grid((nx, n, n), device, (x0, 0, 0))
        p = torch.stack([x, y, z], -1)
        d = torch.sqrt((x - center[0]) ** 2 + (y - center[1]) ** 2 + (z - center[2]) ** 2)
        out[x0:x0 + nx] = (gain * (1.0 - d / radius) + amplitude * fbm(p / scale, 3, seed)).clamp(0.0, 1.0)
    if levels > 0:
        out = torch.floor(out * levels) / levels
    return out


def water_frame(t, nx=1024, ny=256, nz=1024, speed=8.0, base=128.0, amp=24.0, scale=128.0,
                wet0=288.0, wet1=1024.0, n_frames=16, seed=3, device="cpu", outside=100.0):
    """Frame t of an advected noisy water surface, as a signed distance in voxel units.

    Height h_t(x,z) = base + amp * fbm4(q_t / scale) with q_t = (x,z) - t U (sin 2 pi z/512,
    cos 2 pi x/512); phi = (y - h_t) / sqrt(1 + |grad h_t|^2) inside the wet region
    x < X_t (X_t growing linearly from wet0 to wet1 over the frames), `outside` elsewhere."""
    xs = torch.arange(nx, dtype=torch.float32, device=device)
    zs = torch.arange(nz, dtype=torch.float32, device=device)
    X, Z = torch.meshgrid(xs, zs, indexing="ij")

    def height(X, Z):
        qx = X - t * speed * torch.sin(2 * math.pi * Z / 512.0)
        qz = Z - t * speed * torch.cos(2 * math.pi * X / 512.0)
        p = torch.stack([qx / scale, torch.zeros_like(qx), qz / scale], -1)
        return base + amp * fbm(p, 4, seed)

    h = height(X, Z)
    hx = (height(X + 0.5, Z) - height(X - 0.5, Z))
    hz = (height(X, Z + 0.5) - height(X, Z - 0.5))
    norm = torch.sqrt(1.0 + hx * hx + hz * hz)
    wet = wet0 + (wet1 - wet0) * (t / max(n_frames - 1, 1))
    ys = torch.arange(ny, dtype=torch.float32, device=device)
    phi = (ys[None, :, None] - h[:, None, :]) / norm[:, None, :]
    phi = torch.where((X < wet)[:, None, :], phi, torch.full_like(phi, outside))
    return phi.contiguous()
