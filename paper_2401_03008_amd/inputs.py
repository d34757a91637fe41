"""Seeded synthetic initial data: cell-centred rho, v, p and face-staggered B.

This module holds only the definitions of the test problems.  It performs no
step of the solver (no conversion to conserved variables, no reconstruction,
no flux), so both the GPU path and the CPU oracle can start from the same
inputs.

Layout: numpy float64 arrays of shape (nz, ny, nx), x fastest.  Cell centres
are at ((i+1/2) dx, (j+1/2) dy, (k+1/2) dz); the face array bf[d] holds B_d at
the +d face of each cell, e.g. bf[0][k, j, i] = B_x((i+1) dx, (j+1/2) dy,
(k+1/2) dz).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA_AD = 4.0 / 3.0


def cpa_alfven_speed(rho=1.0, p=1.0, B0=1.0, eta=1.0, gam=GAMMA_AD):
    """Exact speed of the large-amplitude circularly polarised Alfven wave
    (Sec. 4, equation for v_A^2; rho h = rho + gam/(gam-1) p)."""
    rhoh = rho + gam / (gam - 1.0) * p
    a = rhoh + B0 * B0 * (1.0 + eta * eta)
    x = 2.0 * eta * B0 * B0 / a
    return math.sqrt(B0 * B0 / a / (0.5 * (1.0 + math.sqrt(1.0 - x * x))))


def cpa_basis(diagonal: bool):
    """Right-handed orthonormal (X, Y, Z) with X the propagation direction.

    Axis case: X = x.  Diagonal case: X = (1,1,1)/sqrt3, Y = (-1,1,0)/sqrt2,
    Z = X x Y.  The paper rotates the wave onto the box diagonal (Sec. 4);
    any right-handed basis with this X is an equally exact wave."""
    if not diagonal:
        return np.eye(3)
    X = np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0)
    Y = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0)
    Z = np.cross(X, Y)
    return np.stack([X, Y, Z])


def cpa_wavevector(diagonal: bool, L=(1.0, 1.0, 1.0)):
    if diagonal:
        return np.array([2 * math.pi / L[0], 2 * math.pi / L[1], 2 * math.pi / L[2]])
    return np.array([2 * math.pi / L[0], 0.0, 0.0])


def cpa_period(diagonal: bool, rho=1.0, p=1.0, B0=1.0, eta=1.0, gam=GAMMA_AD,
               L=(1.0, 1.0, 1.0)):
    """T = 2 pi / (|k| v_A)."""
    k = np.linalg.norm(cpa_wavevector(diagonal, L))
    return 2 * math.pi / (k * cpa_alfven_speed(rho, p, B0, eta, gam))


def _fields_at(x, y, z, t, diagonal, rho, p, B0, eta, gam, L, xp=np):
    XYZ = cpa_basis(diagonal)
    kv = cpa_wavevector(diagonal, L)
    va = cpa_alfven_speed(rho, p, B0, eta, gam)
    phi = kv[0] * x + kv[1] * y + kv[2] * z - float(np.linalg.norm(kv)) * va * t
    c, s = xp.cos(phi), xp.sin(phi)
    B = [B0 * XYZ[0][d] + eta * B0 * (c * XYZ[1][d] + s * XYZ[2][d]) for d in range(3)]
    v = [-va * eta * (c * XYZ[1][d] + s * XYZ[2][d]) for d in range(3)]
    return v, B


def cpa(n, diagonal=True, t=0.0, rho=1.0, p=1.0, B0=1.0, eta=1.0, gam=GAMMA_AD,
        L=(1.0, 1.0, 1.0), device=None):
    """Exact CPA wave at time t on an (nz, ny, nx) grid.

    n is an int (cube) or (nx, ny, nz).  Returns (prim5, bf, Bc): prim5 =
    [rho, vx, vy, vz, p] at cell centres, bf = face B point-sampled at face
    centres, Bc = the exact B at cell centres (for error measurement).
    numpy float64 arrays, or torch float64 tensors on `device` if given."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    dx, dy, dz = L[0] / nx, L[1] / ny, L[2] / nz
    if device is None:
        xp, ar = np, (lambda m, o, h: (np.arange(m) + o) * h)
        mesh = lambda a, b, c: np.meshgrid(a, b, c, indexing="ij")
        full = lambda v: np.full((nz, ny, nx), float(v))
        cont = np.ascontiguousarray
    else:
        import torch
        xp = torch
        ar = lambda m, o, h: (torch.arange(m, dtype=torch.float64, device=device) + o) * h
        mesh = lambda a, b, c: torch.meshgrid(a, b, c, indexing="ij")
        full = lambda v: torch.full((nz, ny, nx), float(v), dtype=torch.float64, device=device)
        cont = lambda a: a.contiguous()
    xc, yc, zc = ar(nx, 0.5, dx), ar(ny, 0.5, dy), ar(nz, 0.5, dz)
    xf, yf, zf = ar(nx, 1.0, dx), ar(ny, 1.0, dy), ar(nz, 1.0, dz)
    Z, Y, X = mesh(zc, yc, xc)
    v, Bc = _fields_at(X, Y, Z, t, diagonal, rho, p, B0, eta, gam, L, xp)
    del X, Y, Z
    prim5 = [full(rho), cont(v[0]), cont(v[1]), cont(v[2]), full(p)]
    del v
    bf = []
    for d in range(3):
        coords = [xc, yc, zc]
        coords[d] = [xf, yf, zf][d]
        Zf, Yf, Xf = mesh(coords[2], coords[1], coords[0])
        _, Bd = _fields_at(Xf, Yf, Zf, t, diagonal, rho, p, B0, eta, gam, L, xp)
        bf.append(cont(Bd[d]))
        del Zf, Yf, Xf, Bd
    return prim5, bf, [cont(b) for b in Bc]


def turbulence(n, sigma0=10.0, beta0=0.1, B0=1.0, nmodes=16, kmax=2, gamma_max=5.0,
               seed=20240103, L=(1.0, 1.0, 1.0), device=None):
    """Decaying Alfvenic turbulence, 3D synthetic stand-in for the paper's 2D
    random-phase set-up (Sec. 5): uniform B0 along z, rho0 = B0^2/sigma0,
    p0 = beta0 B0^2 / 2, plus nmodes random-phase transverse modes with
    integer wave numbers in [-kmax, kmax]^3, (n_x, n_y) != 0, one of each +-k
    pair.

    Magnetic perturbation: edge vector potential A_z = sum sin(k.x + phi_B) /
    |k_perp| at (x_{i+1/2}, y_{j+1/2}, z_k); face B = its discrete curl
    (B_x = dA_z/dy, B_y = -dA_z/dx), so div B vanishes to round-off; A is
    rescaled so that max |dB| = B0.  Velocity: 4-velocity u = -sum e_k
    cos(k.x + phi_v), e_k = (k_hat x z)/|k_hat x z|, rescaled so that
    max Gamma = gamma_max, v = u / sqrt(1 + u^2).

    Returns (prim5, bf): numpy arrays, or torch float64 tensors on `device`.
    The modes and phases come from numpy's default_rng(seed) either way."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    rng = np.random.default_rng(seed)
    cand = []
    for a in range(-kmax, kmax + 1):
        for b in range(-kmax, kmax + 1):
            for c in range(-kmax, kmax + 1):
                if a > 0 or (a == 0 and b > 0):
                    cand.append((a, b, c))
    pick = rng.choice(len(cand), size=nmodes, replace=False)
    modes = [cand[i] for i in sorted(pick)]
    phiB = rng.uniform(0, 2 * math.pi, nmodes)
    phiv = rng.uniform(0, 2 * math.pi, nmodes)

    if device is None:
        xp = np
        ar = lambda m, o, h: (np.arange(m) + o) * h
        mesh = lambda a, b, c: np.meshgrid(a, b, c, indexing="ij")
        zeros = lambda: np.zeros((nz, ny, nx))
        full = lambda v: np.full((nz, ny, nx), float(v))
        roll = lambda a, ax: np.roll(a, 1, axis=ax)
        cont = np.ascontiguousarray
        amax = lambda a: float(a.max())
    else:
        import torch
        xp = torch
        ar = lambda m, o, h: (torch.arange(m, dtype=torch.float64, device=device) + o) * h
        mesh = lambda a, b, c: torch.meshgrid(a, b, c, indexing="ij")
        zeros = lambda: torch.zeros((nz, ny, nx), dtype=torch.float64, device=device)
        full = lambda v: torch.full((nz, ny, nx), float(v), dtype=torch.float64, device=device)
        roll = lambda a, ax: torch.roll(a, 1, dims=ax)
        cont = lambda a: a.contiguous()
        amax = lambda a: float(a.max().item())
    dx, dy, dz = L[0] / nx, L[1] / ny, L[2] / nz
    xc, yc, zc = ar(nx, 0.5, dx), ar(ny, 0.5, dy), ar(nz, 0.5, dz)
    xf, yf = ar(nx, 1.0, dx), ar(ny, 1.0, dy)

    A = zeros()
    ux, uy = zeros(), zeros()
    Ze, Ye, Xe = mesh(zc, yf, xf)
    Zc, Yc, Xc = mesh(zc, yc, xc)
    for (a, b, c), pB, pv in zip(modes, phiB, phiv):
        k = [2 * math.pi * a / L[0], 2 * math.pi * b / L[1], 2 * math.pi * c / L[2]]
        kp = math.hypot(k[0], k[1])
        A += xp.sin(k[0] * Xe + k[1] * Ye + k[2] * Ze + float(pB)) / kp
        e = (k[1] / kp, -k[0] / kp)
        cv = xp.cos(k[0] * Xc + k[1] * Yc + k[2] * Zc + float(pv))
        ux -= e[0] * cv
        uy -= e[1] * cv
    del Ze, Ye, Xe, Zc, Yc, Xc
    # face B from the discrete curl of A_z (A at (i+1/2, j+1/2, k))
    bx = (A - roll(A, 1)) / dy
    by = -(A - roll(A, 2)) / dx
    del A
    # rescale so that max |dB| at cell centres (face averages) equals B0
    bxc = 0.5 * (bx + roll(bx, 2))
    byc = 0.5 * (by + roll(by, 1))
    scale = B0 / math.sqrt(amax(bxc ** 2 + byc ** 2))
    del bxc, byc
    bx = bx * scale
    by = by * scale
    umax = math.sqrt(gamma_max ** 2 - 1.0)
    us = umax / math.sqrt(amax(ux ** 2 + uy ** 2))
    ux = ux * us
    uy = uy * us
    lor = xp.sqrt(1.0 + ux ** 2 + uy ** 2)
    rho0 = B0 * B0 / sigma0
    p0 = 0.5 * beta0 * B0 * B0
    prim5 = [full(rho0), cont(ux / lor), cont(uy / lor), zeros(), full(p0)]
    return prim5, [cont(bx), cont(by), full(B0)]


def turbulence2d_modes(kmax=4):
    """Wave vectors (kx, ky) of the 2D set-up (Sec. 5): kx in 0..kmax, ky in
    -kmax..kmax, 1 <= |k| <= kmax (the disk of radius kmax), one of each +-k
    pair (kx = 0 keeps ky > 0)."""
    out = []
    for a in range(0, kmax + 1):
        for b in range(-kmax, kmax + 1):
            if (a == 0 and b <= 0) or a * a + b * b > kmax * kmax:
                continue
            out.append((a, b))
    return out


def turbulence2d(n, rho0=1.0, sigma0=100.0, beta0=1.0, eta_rms=0.25, kmax=4, seed=20240103,
                 device=None):
    """The 2D (2.5D) Alfvenic turbulence set-up of Sec. 5 on an n x n x 1 box
    of side 2 pi (the z direction uniform, depth 2 pi): static homogeneous
    rho0, B0 = sqrt(sigma0 rho0) along z, p0 = beta0 B0^2 / 2, plus in-plane
    fluctuations dv = A_v sum (k x z)/k cos(k.x + phi_v(k)) and
    dB = A_B sum (k x z)/k cos(k.x + phi_B(k)) over turbulence2d_modes(kmax),
    with independent uniform random phases (numpy default_rng(seed); the
    paper's phases are not published).  dB is the discrete curl of the edge
    potential A_z = A_B sum sin(k.x + phi_B)/k, so div B vanishes to
    round-off.  The amplitudes are fixed a posteriori so that the box means
    <|dv|>/v_A and <|dB|>/B0 (dB at the centres, face averages) equal eta_rms,
    with v_A = B0 / sqrt(rho0 + 4 p0 + B0^2) (gamma = 4/3).

    Returns (prim5, bf, L): numpy arrays (or torch float64 tensors on
    `device`) of shape (1, n, n) and the box lengths (2 pi, 2 pi, 2 pi)."""
    modes = turbulence2d_modes(kmax)
    rng = np.random.default_rng(seed)
    phiv = rng.uniform(0, 2 * math.pi, len(modes))
    phiB = rng.uniform(0, 2 * math.pi, len(modes))
    L = 2 * math.pi
    h = L / n
    if device is None:
        xp = np
        ar = lambda o: (np.arange(n) + o) * h
        mesh = lambda a, b: np.meshgrid(a, b, indexing="ij")
        zeros = lambda: np.zeros((1, n, n))
        roll = lambda a, ax: np.roll(a, 1, axis=ax)
        mean = lambda a: float(a.mean())
    else:
        import torch
        xp = torch
        ar = lambda o: (torch.arange(n, dtype=torch.float64, device=device) + o) * h
        mesh = lambda a, b: torch.meshgrid(a, b, indexing="ij")
        zeros = lambda: torch.zeros((1, n, n), dtype=torch.float64, device=device)
        roll = lambda a, ax: torch.roll(a, 1, dims=ax)
        mean = lambda a: float(a.mean().item())
    Yc, Xc = mesh(ar(0.5), ar(0.5))
    Ye, Xe = mesh(ar(1.0), ar(1.0))
    A, vx, vy = zeros(), zeros(), zeros()
    for (a, b), pv, pb in zip(modes, phiv, phiB):
        k = math.hypot(a, b)
        A[0] += xp.sin(a * Xe + b * Ye + float(pb)) / k
        c = xp.cos(a * Xc + b * Yc + float(pv))
        vx[0] += (b / k) * c
        vy[0] -= (a / k) * c
    del Xc, Yc, Xe, Ye
    # face B from the discrete curl of A_z at (x_{i+1/2}, y_{j+1/2})
    bx = (A - roll(A, 1)) / h
    by = -(A - roll(A, 2)) / h
    del A
    B0 = math.sqrt(sigma0 * rho0)
    p0 = 0.5 * beta0 * B0 * B0
    va = B0 / math.sqrt(rho0 + 4.0 * p0 + B0 * B0)
    bxc = 0.5 * (bx + roll(bx, 2))
    byc = 0.5 * (by + roll(by, 1))
    sB = eta_rms * B0 / mean(xp.sqrt(bxc ** 2 + byc ** 2))
    sv = eta_rms * va / mean(xp.sqrt(vx ** 2 + vy ** 2))
    del bxc, byc
    full = lambda v: zeros() + float(v)
    prim5 = [full(rho0), vx * sv, vy * sv, zeros(), full(p0)]
    bf = [bx * sB, by * sB, full(B0)]
    if device is None:
        prim5 = [np.ascontiguousarray(q) for q in prim5]
        bf = [np.ascontiguousarray(q) for q in bf]
    else:
        prim5 = [q.contiguous() for q in prim5]
        bf = [q.contiguous() for q in bf]
    return prim5, bf, (L, L, L)
