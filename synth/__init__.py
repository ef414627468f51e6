"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no step of the rendering method: it only builds emissivity
and velocity fields (and view lists) in the caller's layout

    j    [M][nz][ny][nx]       rest-frame emissivity at the reference frequency
    beta [M][nz][ny][nx][3]    velocity in units of c
    times[M]                   strictly increasing epoch times

from seeded random numbers (numpy's PCG64 via ``default_rng``).  The large
jet-like stacks are filled on the device by ``synth/jetgen.hip`` from
parameters drawn here, so that 10-170 GB stacks never pass through host memory.

Workload recipes (cells are unit cubes, cell centres at (i+1/2, j+1/2, k+1/2)):

* ``blobs``  three advected Gaussian blobs (sigma 4 cells, amplitudes
  U[0.5, 2], centres U[16, 48]^3 at t = 0 on a 64^3 grid, moving +0.6 cell per
  unit time along z); beta = (0, 0, 0.6) within 2 sigma of a centre, else 0.
* ``jet``    a cylindrical jet along z (radius 12 cells, Lorentz factor falling
  from the spine value to 1.2 at the edge), lognormal (sigma 0.5) turbulence
  from 64 advected Fourier modes (wavelengths U[4, 32] cells), rho^1.5
  emissivity (x0.01 outside the jet) and propagating knots (beta 0.98,
  Gaussian brightening of width 6 cells, 12-cell velocity region).
* ``twin_ejecta``  two anti-parallel homogeneous ejecta, spheres of radius R
  in their rest frames, contracted by 1/Gamma along the motion (the mock of the
  paper's Sec. 3), with cell coverage sampled on a sub-grid.
* ``random``  uniform random emissivity and velocities (|beta| <= beta_max).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_GEN_SRC = os.path.join(_HERE, "jetgen.hip")
_GEN_LIB = os.path.join(_HERE, "libsynth.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# --------------------------------------------------------------------------
# small host-side recipes
# --------------------------------------------------------------------------

def random_stack(dims, n_epochs, seed, beta_max=0.9, times=None, dtype=np.float64,
                 j_range=(0.0, 1.0)):
    """Uniform random fields: j ~ U[j_range], beta uniform in the ball of radius
    beta_max (direction isotropic, |beta| = beta_max * U^(1/3))."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    shape = (n_epochs, nz, ny, nx)
    j = rng.uniform(j_range[0], j_range[1], size=shape)
    d = rng.normal(size=shape + (3,))
    d /= np.linalg.norm(d, axis=-1, keepdims=True) + 1e-300
    r = beta_max * rng.uniform(0, 1, size=shape) ** (1.0 / 3.0)
    beta = d * r[..., None]
    if times is None:
        times = np.cumsum(rng.uniform(0.5, 2.0, size=n_epochs)) - 1.0
    return j.astype(dtype), beta.astype(dtype), np.asarray(times, dtype=np.float64)


def blobs(seed=1, n=64, times=(0.0, 1.0, 2.0, 3.0), sigma=4.0, speed=0.6, n_blobs=3):
    """The 64^3 three-blob recipe (FP64)."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(16.0, 48.0, size=(n_blobs, 3)) * (n / 64.0)
    amps = rng.uniform(0.5, 2.0, size=n_blobs)
    times = np.asarray(times, dtype=np.float64)
    c = np.arange(n) + 0.5
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    M = len(times)
    j = np.zeros((M, n, n, n))
    beta = np.zeros((M, n, n, n, 3))
    for m, t in enumerate(times):
        inside = np.zeros((n, n, n), dtype=bool)
        for b in range(n_blobs):
            cx, cy, cz = centres[b]
            cz = cz + speed * t
            r2 = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2
            j[m] += amps[b] * np.exp(-r2 / (2 * sigma * sigma))
            inside |= r2 <= (2 * sigma) ** 2
        beta[m, inside, 2] = speed
    return j, beta, times


def twin_ejecta(dims=(28, 28, 84), radius=6.0, gamma=2.0, times=None, t_centre=0.0, sub=4,
                axis_sep=8.0, jval=1.0):
    """Two homogeneous ejecta moving along +z and -z from the grid centre C.

    Each is a sphere of ``radius`` cells in its rest frame; in the lab frame it
    is contracted by 1/gamma along z.  At time t the advancing one is centred at
    C + (axis_sep + v (t - t_centre)) z_hat and the receding one at the mirror
    point, so the pair is point-symmetric about C at every epoch.  Each
    ejectum is kept to its own half-space (z >= C_z or z < C_z), so the two never
    share a cell.  The emissivity of a cell is jval times the fraction of its
    volume inside the spheroid, sampled on a sub^3 lattice of points.
    """
    beta = math.sqrt(1.0 - 1.0 / (gamma * gamma))
    if times is None:
        times = np.arange(-12.0, 36.0 + 1e-9, 1.0)
    times = np.asarray(times, dtype=np.float64)
    nx, ny, nz = dims
    M = len(times)
    Cx, Cy, Cz = 0.5 * nx, 0.5 * ny, 0.5 * nz
    j = np.zeros((M, nz, ny, nx))
    bvec = np.zeros((M, nz, ny, nx, 3))
    off = (np.arange(sub) + 0.5) / sub
    rz = radius / gamma
    x0, x1 = int(max(0, math.floor(Cx - radius - 1))), int(min(nx, math.ceil(Cx + radius + 1)))
    y0, y1 = int(max(0, math.floor(Cy - radius - 1))), int(min(ny, math.ceil(Cy + radius + 1)))
    xi, yi = np.arange(x0, x1), np.arange(y0, y1)
    px = (xi[:, None] + off[None, :]).reshape(-1)
    py = (yi[:, None] + off[None, :]).reshape(-1)
    for m, t in enumerate(times):
        zc = axis_sep + beta * (t - t_centre)
        for sgn in (+1, -1):
            cz = Cz + sgn * zc
            z0 = int(max(0, math.floor(cz - rz - 1)))
            z1 = int(min(nz, math.ceil(cz + rz + 1)))
            if sgn > 0:
                z0 = max(z0, int(math.ceil(Cz)))
            else:
                z1 = min(z1, int(math.floor(Cz)))
            if z0 >= z1:
                continue
            zi = np.arange(z0, z1)
            pz = (zi[:, None] + off[None, :]).reshape(-1)
            Z, Y, X = np.meshgrid(pz, py, px, indexing="ij")
            inside = ((X - Cx) ** 2 + (Y - Cy) ** 2) / radius ** 2 + ((Z - cz) / rz) ** 2 <= 1.0
            cov = inside.reshape(len(zi), sub, len(yi), sub, len(xi), sub).mean(axis=(1, 3, 5))
            j[m, z0:z1, y0:y1, x0:x1] = jval * cov
            blk = bvec[m, z0:z1, y0:y1, x0:x1]
            blk[cov > 0, 2] = sgn * beta
    return j, bvec, times


def isotropic_views(n, seed, sizes=(128, 256, 512, 1024)):
    """n views with cos(theta) ~ U[-1, 1], phi ~ U[0, 360) and an image side
    drawn uniformly from ``sizes``: list of (theta_deg, phi_deg, side)."""
    rng = np.random.default_rng(seed)
    ct = rng.uniform(-1.0, 1.0, size=n)
    ph = rng.uniform(0.0, 360.0, size=n)
    side = rng.choice(np.asarray(sizes), size=n)
    return [(math.degrees(math.acos(c)), p, int(s)) for c, p, s in zip(ct, ph, side)]


def diag(dims):
    return math.sqrt(sum(float(d) ** 2 for d in dims))


def jet_times(dims, n_epochs):
    """t_m = -L/2 + m L / (M - 1) with L the grid diagonal: with t_obs = 0 the
    window covers every cell at every orientation."""
    L = diag(dims)
    return -0.5 * L + np.arange(n_epochs) * (L / (n_epochs - 1))


# --------------------------------------------------------------------------
# jet recipe: parameters on the host, fields on the device
# --------------------------------------------------------------------------

class JetParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("n_modes", ctypes.c_int), ("n_knots", ctypes.c_int),
                ("gamma_spine", ctypes.c_float), ("r_jet", ctypes.c_float),
                ("knot_beta", ctypes.c_float), ("knot_radius", ctypes.c_float),
                ("knot_sigma", ctypes.c_float), ("knot_amp", ctypes.c_float),
                ("turb_speed", ctypes.c_float), ("outside", ctypes.c_float),
                ("k", ctypes.c_float * (64 * 3)), ("phase", ctypes.c_float * 64),
                ("knot_z0", ctypes.c_float * 16),
                ("z_begin", ctypes.c_int), ("z_count", ctypes.c_int)]


def jet_params(dims, seed, gamma_spine=5.0, n_knots=4, n_modes=64):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    p = JetParams()
    p.nx, p.ny, p.nz = nx, ny, nz
    p.n_modes, p.n_knots = n_modes, n_knots
    p.gamma_spine, p.r_jet = gamma_spine, 12.0
    p.knot_beta, p.knot_radius, p.knot_sigma, p.knot_amp = 0.98, 12.0, 6.0, 4.0
    p.turb_speed, p.outside = 0.5, 0.01
    lam = rng.uniform(4.0, 32.0, size=n_modes)
    d = rng.normal(size=(n_modes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    k = d * (2 * math.pi / lam)[:, None]
    p.k[:] = [float(x) for x in k.reshape(-1)] + [0.0] * (192 - 3 * n_modes)
    p.phase[:] = [float(x) for x in rng.uniform(0, 2 * math.pi, size=n_modes)] + [0.0] * (64 - n_modes)
    z0 = rng.uniform(0, nz, size=n_knots)
    p.knot_z0[:] = [float(x) for x in z0] + [0.0] * (16 - n_knots)
    p.z_begin, p.z_count = 0, nz
    return p


def build(force: bool = True) -> str:
    """Compile the device generator into ``synth/libsynth.so``."""
    if force or not os.path.exists(_GEN_LIB):
        tmp = _GEN_LIB + ".tmp"
        subprocess.check_call([HIPCC] + HIP_FLAGS + ["-o", tmp, _GEN_SRC])
        os.replace(tmp, _GEN_LIB)
    return _GEN_LIB


_glib = None


def _gen():
    global _glib
    if _glib is None:
        if not os.path.exists(_GEN_LIB):
            raise RuntimeError("synth/libsynth.so is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_GEN_LIB)
        lib.synth_jet_fill.restype = ctypes.c_int
        lib.synth_jet_fill.argtypes = [ctypes.POINTER(JetParams), ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]
        _glib = lib
    return _glib


def jet_fill_device(params: JetParams, times, j_ptr: int, beta_ptr: int, stream: int = 0):
    """Fill device arrays j [M][nz][ny][nx] and beta [M][nz][ny][nx][3] (float32)
    with the jet recipe at the given epoch times."""
    t = np.ascontiguousarray(times, dtype=np.float64)
    rc = _gen().synth_jet_fill(ctypes.byref(params), len(t),
                               t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.c_void_p(j_ptr), ctypes.c_void_p(beta_ptr),
                               ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError(f"synth_jet_fill failed ({rc})")


def jet_torch(dims, n_epochs, seed, gamma_spine=5.0, n_knots=4, device="cuda", times=None,
              z_slab=None):
    """Convenience: allocate float32 torch tensors on the device and fill them.
    z_slab=(z0, nz_slab) fills only those z-layers of the domain `dims`, with
    the same values the whole domain holds there."""
    import torch
    nx, ny, nz = dims
    if times is None:
        times = jet_times(dims, n_epochs)
    p = jet_params(dims, seed, gamma_spine=gamma_spine, n_knots=n_knots)
    if z_slab is not None:
        p.z_begin, p.z_count = int(z_slab[0]), int(z_slab[1])
        nz = p.z_count
    j = torch.empty((n_epochs, nz, ny, nx), dtype=torch.float32, device=device)
    b = torch.empty((n_epochs, nz, ny, nx, 3), dtype=torch.float32, device=device)
    jet_fill_device(p, times, j.data_ptr(), b.data_ptr(),
                    torch.cuda.current_stream().cuda_stream)
    return j, b, np.asarray(times, dtype=np.float64)


# --------------------------------------------------------------------------
# host-side storage rounding (what a 16-bit stack holds), numpy only
# --------------------------------------------------------------------------

def round_f16(x):
    """Round-to-nearest-even to IEEE binary16 and back to float32."""
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float32)


def round_bf16(x):
    """Round-to-nearest-even to bfloat16 and back to float32 (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def to_bf16_bits(x):
    """bfloat16 bit patterns (uint16) of float32 values, rounded to nearest even."""
    return (round_bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def to_f16(x):
    """IEEE binary16 values of float32 inputs (numpy rounds to nearest even)."""
    return np.asarray(x, dtype=np.float32).astype(np.float16)
