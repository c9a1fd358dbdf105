"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random parameters and evaluates analytic fields; it holds none of the tracking method's
arithmetic.  Both the HIP path and the oracle consume the arrays it returns.

Moving-blob fields stand in for the paper's application datasets (flow, fusion blobs, turbulent vortices, Sec. 4.6),
which are not available.  Recipe (drawn with numpy's PCG64, vectorised over the K blobs, in this order):
sign = -1 where random(K) < 0.5 else +1; amplitude A ~ U(0.5, 1.5); sigma ~ U(lo, hi); centre ~ U(0, n_a) per axis
(x, then y, then z); velocity ~ U(-v, v) per axis; then, if any, the noise array from the same generator.  Values are
evaluated in float64, blob by blob in k order, and cast to float32.  Each blob is evaluated on a window of +-ceil(8
sigma) cells around its centre (beyond it a term is below 1.3e-14 of its amplitude).

Analytic test fields from the paper: the moving minimum (Sec. 4.5, Eq. 3-4) and the spiral woven function (Sec. 4.5,
Eq. 5).
"""
import math

import numpy as np


def _blob_params(rng, K, dims_sp, sigma, vmax):
    sign = np.where(rng.random(K) < 0.5, -1.0, 1.0)
    amp = rng.uniform(0.5, 1.5, K)
    sig = rng.uniform(sigma[0], sigma[1], K)
    centre = np.stack([rng.uniform(0.0, float(N), K) for N in dims_sp], axis=1)
    if np.isscalar(vmax) or len(np.atleast_1d(vmax)) == 1:
        vel = np.stack([rng.uniform(-float(vmax), float(vmax), K) for _ in dims_sp], axis=1)
    else:
        vel = np.stack([rng.uniform(-float(v), float(v), K) for v in vmax], axis=1)
    return sign, amp, sig, centre, vel


def _windows(c, s, N):
    w = int(math.ceil(8.0 * s))
    lo = max(0, int(math.floor(c)) - w)
    hi = min(N, int(math.floor(c)) + w + 2)
    return lo, hi


def moving_gaussians_2d(nx, ny, nt, K, sigma=(4.0, 10.0), vmax=1.0, seed=0, noise_std=0.0, device=None):
    """f[t][y][x] = sum_k s_k A_k exp(-|x - c_k - v_k t|^2 / (2 sigma_k^2)) (+ iid N(0, noise_std) noise).
    With a torch device (and no noise) the same float64 evaluation runs there and a float32 numpy array returns."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sign, amp, sig, centre, vel = _blob_params(rng, K, (nx, ny), sigma, vmax)
    if device is not None and noise_std == 0:
        return _gaussians_2d_torch(nx, ny, nt, K, sign, amp, sig, centre, vel, device)
    f = np.zeros((nt, ny, nx), np.float64)
    for t in range(nt):
        plane = f[t]
        for k in range(K):
            cx = centre[k, 0] + vel[k, 0] * t
            cy = centre[k, 1] + vel[k, 1] * t
            x0, x1 = _windows(cx, sig[k], nx)
            y0, y1 = _windows(cy, sig[k], ny)
            if x0 >= x1 or y0 >= y1:
                continue
            inv = 1.0 / (2.0 * sig[k] * sig[k])
            ex = np.exp(-((np.arange(x0, x1) - cx) ** 2) * inv)
            ey = np.exp(-((np.arange(y0, y1) - cy) ** 2) * inv)
            plane[y0:y1, x0:x1] += (sign[k] * amp[k]) * np.outer(ey, ex)
    if noise_std > 0:
        f += rng.normal(0.0, noise_std, size=f.shape)
    return f.astype(np.float32)


def moving_gaussians_3d(nx, ny, nz, nt, K, sigma=(6.0, 16.0), vmax=1.0, seed=2, device=None):
    """3D analogue, f[t][z][y][x], separable window per blob.  With a torch device the same float64 evaluation runs
    there (the large 3D workload would take minutes in numpy); the float32 result is returned as a numpy array."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sign, amp, sig, centre, vel = _blob_params(rng, K, (nx, ny, nz), sigma, vmax)
    if device is not None:
        return _gaussians_3d_torch(nx, ny, nz, nt, K, sign, amp, sig, centre, vel, device)
    f = np.zeros((nt, nz, ny, nx), np.float64)
    for t in range(nt):
        vol = f[t]
        for k in range(K):
            c = [centre[k, a] + vel[k, a] * t for a in range(3)]
            rx = _windows(c[0], sig[k], nx)
            ry = _windows(c[1], sig[k], ny)
            rz = _windows(c[2], sig[k], nz)
            if rx[0] >= rx[1] or ry[0] >= ry[1] or rz[0] >= rz[1]:
                continue
            inv = 1.0 / (2.0 * sig[k] * sig[k])
            ex = np.exp(-((np.arange(*rx) - c[0]) ** 2) * inv)
            ey = np.exp(-((np.arange(*ry) - c[1]) ** 2) * inv)
            ez = np.exp(-((np.arange(*rz) - c[2]) ** 2) * inv)
            vol[rz[0]:rz[1], ry[0]:ry[1], rx[0]:rx[1]] += (sign[k] * amp[k]) * (
                ez[:, None, None] * ey[None, :, None] * ex[None, None, :])
    return f.astype(np.float32)


def _gaussians_2d_torch(nx, ny, nt, K, sign, amp, sig, centre, vel, device):
    import torch
    out = np.empty((nt, ny, nx), np.float32)
    for t in range(nt):
        plane = torch.zeros((ny, nx), dtype=torch.float64, device=device)
        for k in range(K):
            cx = centre[k, 0] + vel[k, 0] * t
            cy = centre[k, 1] + vel[k, 1] * t
            x0, x1 = _windows(cx, sig[k], nx)
            y0, y1 = _windows(cy, sig[k], ny)
            if x0 >= x1 or y0 >= y1:
                continue
            inv = 1.0 / (2.0 * sig[k] * sig[k])
            ex = torch.exp(-((torch.arange(x0, x1, dtype=torch.float64, device=device) - cx) ** 2) * inv)
            ey = torch.exp(-((torch.arange(y0, y1, dtype=torch.float64, device=device) - cy) ** 2) * inv)
            plane[y0:y1, x0:x1] += (float(sign[k]) * float(amp[k])) * (ey[:, None] * ex[None, :])
        out[t] = plane.to(torch.float32).cpu().numpy()
    return out


def _gaussians_3d_torch(nx, ny, nz, nt, K, sign, amp, sig, centre, vel, device):
    import torch
    out = np.empty((nt, nz, ny, nx), np.float32)
    for t in range(nt):
        vol = torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
        for k in range(K):
            c = [centre[k, a] + vel[k, a] * t for a in range(3)]
            rx = _windows(c[0], sig[k], nx)
            ry = _windows(c[1], sig[k], ny)
            rz = _windows(c[2], sig[k], nz)
            if rx[0] >= rx[1] or ry[0] >= ry[1] or rz[0] >= rz[1]:
                continue
            inv = 1.0 / (2.0 * sig[k] * sig[k])
            ex = torch.exp(-((torch.arange(*rx, dtype=torch.float64, device=device) - c[0]) ** 2) * inv)
            ey = torch.exp(-((torch.arange(*ry, dtype=torch.float64, device=device) - c[1]) ** 2) * inv)
            ez = torch.exp(-((torch.arange(*rz, dtype=torch.float64, device=device) - c[2]) ** 2) * inv)
            vol[rz[0]:rz[1], ry[0]:ry[1], rx[0]:rx[1]] += (float(sign[k]) * float(amp[k])) * (
                ez[:, None, None] * ey[None, :, None] * ex[None, None, :])
        out[t] = vol.to(torch.float32).cpu().numpy()
    return out


def vortex_sources_2d(nx, ny, nt, K, sigma=(16.0, 48.0), vmax=2.0, seed=4, device=None):
    """Vector field u[t][c][y][x]: half the blobs contribute grad G (sources/sinks), half the rotated gradient
    (-dG/dy, dG/dx) (vortices), G = s A exp(-r^2 / (2 sigma^2)); derivatives are analytic.  The blob kind is drawn
    after the shared parameters (kind = vortex where random(K) < 0.5)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sign, amp, sig, centre, vel = _blob_params(rng, K, (nx, ny), sigma, vmax)
    vortex = rng.random(K) < 0.5
    if device is not None:
        return _vortex_sources_torch(nx, ny, nt, K, sign, amp, sig, centre, vel, vortex, device)
    u = np.zeros((nt, 2, ny, nx), np.float64)
    for t in range(nt):
        for k in range(K):
            cx = centre[k, 0] + vel[k, 0] * t
            cy = centre[k, 1] + vel[k, 1] * t
            x0, x1 = _windows(cx, sig[k], nx)
            y0, y1 = _windows(cy, sig[k], ny)
            if x0 >= x1 or y0 >= y1:
                continue
            inv = 1.0 / (2.0 * sig[k] * sig[k])
            dx = np.arange(x0, x1) - cx
            dy = np.arange(y0, y1) - cy
            G = (sign[k] * amp[k]) * np.outer(np.exp(-(dy ** 2) * inv), np.exp(-(dx ** 2) * inv))
            gx = -G * (dx[None, :] / (sig[k] * sig[k]))
            gy = -G * (dy[:, None] / (sig[k] * sig[k]))
            if vortex[k]:
                u[t, 0, y0:y1, x0:x1] += -gy
                u[t, 1, y0:y1, x0:x1] += gx
            else:
                u[t, 0, y0:y1, x0:x1] += gx
                u[t, 1, y0:y1, x0:x1] += gy
    return u.astype(np.float32)


def _vortex_sources_torch(nx, ny, nt, K, sign, amp, sig, centre, vel, vortex, device):
    import torch
    out = np.empty((nt, 2, ny, nx), np.float32)
    for t in range(nt):
        u = torch.zeros((2, ny, nx), dtype=torch.float64, device=device)
        for k in range(K):
            cx = centre[k, 0] + vel[k, 0] * t
            cy = centre[k, 1] + vel[k, 1] * t
            x0, x1 = _windows(cx, sig[k], nx)
            y0, y1 = _windows(cy, sig[k], ny)
            if x0 >= x1 or y0 >= y1:
                continue
            inv = 1.0 / (2.0 * sig[k] * sig[k])
            dx = torch.arange(x0, x1, dtype=torch.float64, device=device) - cx
            dy = torch.arange(y0, y1, dtype=torch.float64, device=device) - cy
            G = (float(sign[k]) * float(amp[k])) * (torch.exp(-(dy ** 2) * inv)[:, None] * torch.exp(-(dx ** 2) * inv)[None, :])
            gx = -G * (dx[None, :] / (sig[k] * sig[k]))
            gy = -G * (dy[:, None] / (sig[k] * sig[k]))
            if vortex[k]:
                u[0, y0:y1, x0:x1] += -gy
                u[1, y0:y1, x0:x1] += gx
            else:
                u[0, y0:y1, x0:x1] += gx
                u[1, y0:y1, x0:x1] += gy
        out[t] = u.to(torch.float32).cpu().numpy()
    return out


def quantise_levels(f, levels=16):
    """Degenerate variant: the whole series mapped affinely onto [0, levels-1] and rounded to integers."""
    f64 = f.astype(np.float64)
    lo, hi = f64.min(), f64.max()
    return np.rint((f64 - lo) / (hi - lo) * (levels - 1)).astype(np.float32)


def batch_series(count=96, seed0=3, size_range=(128, 2048), nt_range=(8, 64), k_range=(16, 512),
                 sigma=(4.0, 10.0), vmax=1.0, shape_only=False, device=None):
    """Many independent 2D series of uneven sizes: series i uses seed seed0 + i; nx, ny ~ round(exp(U(ln lo,
    ln hi))), nt ~ integers in nt_range (inclusive), K = clip(round(512 nx ny / 2048^2), k_range); the blobs are
    drawn after these with the shared recipe."""
    out = []
    for i in range(count):
        rng = np.random.Generator(np.random.PCG64(seed0 + i))
        nx = int(round(math.exp(rng.uniform(math.log(size_range[0]), math.log(size_range[1])))))
        ny = int(round(math.exp(rng.uniform(math.log(size_range[0]), math.log(size_range[1])))))
        nt = int(rng.integers(nt_range[0], nt_range[1] + 1))
        K = int(np.clip(round(512 * nx * ny / 2048.0 ** 2), k_range[0], k_range[1]))
        if shape_only:
            out.append((nx, ny, nt, K))
            continue
        # the blob parameters continue from the same generator
        sign, amp, sig, centre, vel = _blob_params(rng, K, (nx, ny), sigma, vmax)
        if device is not None:
            out.append(_gaussians_2d_torch(nx, ny, nt, K, sign, amp, sig, centre, vel, device))
            continue
        f = np.zeros((nt, ny, nx), np.float64)
        for t in range(nt):
            for k in range(K):
                cx = centre[k, 0] + vel[k, 0] * t
                cy = centre[k, 1] + vel[k, 1] * t
                x0, x1 = _windows(cx, sig[k], nx)
                y0, y1 = _windows(cy, sig[k], ny)
                if x0 >= x1 or y0 >= y1:
                    continue
                inv = 1.0 / (2.0 * sig[k] * sig[k])
                f[t, y0:y1, x0:x1] += (sign[k] * amp[k]) * np.outer(
                    np.exp(-((np.arange(y0, y1) - cy) ** 2) * inv), np.exp(-((np.arange(x0, x1) - cx) ** 2) * inv))
        out.append(f.astype(np.float32))
    return out


def moving_minimum(n, size, x0, direction, nt):
    """Sec. 4.5, Eq. 3: f(x, t) = |x - (x0 + d t)|^2 on a size^n grid (f[t][(z)][y][x]).  With dyadic d and integer
    x0 every value is exact in float32."""
    axes = [np.arange(size, dtype=np.float64)] * n
    grids = np.meshgrid(*axes, indexing="ij")  # grids[a][i_x, i_y, ...]
    out = []
    for t in range(nt):
        s = np.zeros(grids[0].shape)
        for a in range(n):
            s += (grids[a] - (x0[a] + direction[a] * t)) ** 2
        out.append(np.transpose(s, tuple(range(n))[::-1]))
    return np.asarray(out, dtype=np.float32)


def spiral_woven(size, nt, extent, dt):
    """Sec. 4.5, Eq. 5: f = cos(x cos t - y sin t) sin(x sin t + y cos t) on [-extent, extent]^2, f[t][y][x]."""
    xs = np.linspace(-extent, extent, size)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    out = []
    for k in range(nt):
        t = k * dt
        out.append(np.cos(X * np.cos(t) - Y * np.sin(t)) * np.sin(X * np.sin(t) + Y * np.cos(t)))
    return np.asarray(out, dtype=np.float32)


# Named workloads (sizes of the paper-shaped synthetic configurations).
def random_waves_3d(nx, ny, nz, nt, K=8, wavelength=(6.0, 16.0), period=(6.0, 20.0), seed=6):
    """Complex 3D series whose real and imaginary parts are independent sums of K random cosine waves each
    (directions uniform on the sphere, wavelengths and periods in the given ranges, amplitudes U(0.5, 1.5), phases
    uniform); their common zero set is a tangle of moving vortex lines.  Returns float32 [nt][2][nz][ny][nx] (real
    and imaginary planes), evaluated in float64."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.arange(nx, dtype=np.float64)
    Y = np.arange(ny, dtype=np.float64)
    Z = np.arange(nz, dtype=np.float64)
    waves = []
    for part in range(2):
        d = rng.normal(size=(K, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        kv = d * (2 * np.pi / rng.uniform(*wavelength, size=K))[:, None]
        w = 2 * np.pi / rng.uniform(*period, size=K)
        amp = rng.uniform(0.5, 1.5, size=K)
        phi = rng.uniform(0, 2 * np.pi, size=K)
        waves.append((kv, w, amp, phi))
    out = np.zeros((nt, 2, nz, ny, nx), np.float32)
    for t in range(nt):
        for part, (kv, w, amp, phi) in enumerate(waves):
            acc = np.zeros((nz, ny, nx))
            for k in range(K):
                acc += amp[k] * np.cos(kv[k, 2] * Z[:, None, None] + kv[k, 1] * Y[None, :, None]
                                       + kv[k, 0] * X[None, None, :] - w[k] * t + phi[k])
            out[t, part] = acc
    return out


def delaunay_mesh(n_points, extent=10.0, seed=7):
    """Unstructured triangle mesh: the Delaunay triangulation of the square's corners and n_points uniform points in
    [0, extent]^2.  Returns (xy float32 [nv][2], tri int32 [nf][3])."""
    from scipy.spatial import Delaunay
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = np.concatenate([np.array([[0, 0], [extent, 0], [0, extent], [extent, extent]], np.float64),
                          rng.uniform(0, extent, size=(n_points, 2))])
    xy = pts.astype(np.float32)
    tri = Delaunay(xy.astype(np.float64)).simplices.astype(np.int32)
    return xy, tri


def kuhn_grid_mesh(nx, ny):
    """The regular nx x ny grid as a triangle mesh (vertex y * nx + x), each cell split along its (0,0)-(1,1)
    diagonal into the triangles x-then-y and y-then-x."""
    xy = np.array([(x, y) for y in range(ny) for x in range(nx)], np.float32)
    tri = []
    for y in range(ny - 1):
        for x in range(nx - 1):
            v = y * nx + x
            tri.append((v, v + 1, v + nx + 1))
            tri.append((v, v + nx, v + nx + 1))
    return xy, np.array(tri, np.int32)


WORKLOAD_PARAMS = {
    "blobs64": dict(n=2, kind=0, dims=(64, 64, 10), K=8, seed=0),
    "noise1024": dict(n=2, kind=0, dims=(1024, 1024, 100), K=256, seed=1, noise_std=1e-3),
    "blobs3d256": dict(n=3, kind=0, dims=(256, 256, 256, 16), K=512, seed=2),
    "vortex4096": dict(n=2, kind=1, dims=(4096, 4096, 50), K=1024, seed=4),
}


def make(name, nt=None, ny=None, device=None):
    """Generate a named workload (optionally only the first nt steps / ny rows; device: torch device for the 3D
    field's float64 evaluation)."""
    c = WORKLOAD_PARAMS["noise1024" if name == "levels1024" else name]
    if name == "blobs64":
        nx, nyy, ntt = c["dims"]
        return moving_gaussians_2d(nx, ny or nyy, nt or ntt, c["K"], seed=c["seed"])
    if name in ("noise1024", "levels1024"):
        nx, nyy, ntt = c["dims"]
        f = moving_gaussians_2d(nx, ny or nyy, nt or ntt, c["K"], seed=c["seed"], noise_std=c["noise_std"])
        return quantise_levels(f) if name == "levels1024" else f
    if name == "blobs3d256":
        nx, nyy, nz, ntt = c["dims"]
        return moving_gaussians_3d(nx, ny or nyy, nz, nt or ntt, c["K"], seed=c["seed"], device=device)
    if name == "vortex4096":
        nx, nyy, ntt = c["dims"]
        return vortex_sources_2d(nx, ny or nyy, nt or ntt, c["K"], seed=c["seed"], device=device)
    raise KeyError(name)
