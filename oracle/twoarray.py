"""Conventional two-array regularized lattice Boltzmann step in numpy (FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  A second, independent
implementation of what ``lbref.c`` computes, written with whole-array numpy
operations instead of per-node loops, for tiny grids.  It follows the same
passages of the paper: moments (Section 2), incompressible equilibrium
(eq. equil), Hermite-regularized non-equilibrium (Section 3, eq. hermite),
post-collision rewrite (eq. LBexp) and push streaming (eq. pushLB), with Guo's
body-force source and halfway bounce-back; the colour-gradient perturbation
and recolouring of Section 2.1 for two species.

Fields are held as arrays of shape (..., nz, ny, nx).
"""
from __future__ import annotations

import itertools

import numpy as np

CS2 = 1.0 / 3.0

_WEIGHTS = {
    9: {0: 4 / 9, 1: 1 / 9, 2: 1 / 36},
    19: {0: 1 / 3, 1: 1 / 18, 2: 1 / 36},
    27: {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216},
}


def velocity_set(kind: int):
    """(c[Q,3], w[Q], opp[Q]) built from the |c|^2-class weights."""
    D = 2 if kind == 9 else 3
    cs, ws = [], []
    for c in itertools.product((-1, 0, 1), repeat=3):
        if D == 2 and c[2] != 0:
            continue
        c2 = sum(ci * ci for ci in c)
        if c2 in _WEIGHTS[kind]:
            cs.append(c)
            ws.append(_WEIGHTS[kind][c2])
    c = np.array(cs, dtype=np.int64)
    opp = np.array([int(np.where((c == -ci).all(axis=1))[0][0]) for ci in c])
    return c, np.array(ws), opp


def _hermite(c, D, dtype=np.float64):
    """H0, H1[Q,D], H2[Q,D,D], H3[Q,D,D,D] evaluated at the lattice velocities."""
    cd = c[:, :D].astype(dtype)
    I = np.eye(D, dtype=dtype)
    H2 = np.einsum("qa,qb->qab", cd, cd) - CS2 * I
    H3 = (np.einsum("qa,qb,qc->qabc", cd, cd, cd)
          - CS2 * (np.einsum("qa,bc->qabc", cd, I)
                   + np.einsum("qb,ac->qabc", cd, I)
                   + np.einsum("qc,ab->qabc", cd, I)))
    return cd, H2, H3


def _collide(g, c, w, D, tau, rho0, F, order):
    """Regularized collision of every node: g[Q,...] -> g^pc[Q,...]."""
    omega = 1.0 / tau
    cd, H2, H3 = _hermite(c, D, g.dtype)
    wq = w.astype(g.dtype).reshape((-1,) + (1,) * (g.ndim - 1))
    rho = g.sum(axis=0)
    j = np.einsum("qa,q...->a...", cd, g)
    Fv = np.asarray(F, dtype=g.dtype)
    if Fv.ndim == 1:  # one constant force, else a force field F[alpha, ...]
        Fv = Fv[:D].reshape((D,) + (1,) * (g.ndim - 1))
    else:
        Fv = Fv[:D]
    u = (j + 0.5 * Fv) / rho0
    uu = np.einsum("a...,b...->ab...", u, u)
    cu = np.einsum("qa,a...->q...", cd, u)
    feq = wq * (rho[None] + rho0 * (cu / CS2 + np.einsum("qab,ab...->q...", H2, uu) / (2 * CS2**2)))
    if order >= 3:
        uuu = np.einsum("a...,b...,c...->abc...", u, u, u)
        feq = feq + wq * rho0 * np.einsum("qabc,abc...->q...", H3, uuu) / (6 * CS2**3)
    fneq = g - feq
    a1 = np.einsum("qa,q...->a...", cd, fneq)
    Pi = np.einsum("qab,q...->ab...", np.einsum("qa,qb->qab", cd, cd), fneq)
    fhat = wq * (np.einsum("qa,a...->q...", cd, a1) / CS2
                 + np.einsum("qab,ab...->q...", H2, Pi) / (2 * CS2**2))
    if order >= 3:
        a3 = (np.einsum("a...,bc...->abc...", u, Pi) + np.einsum("b...,ac...->abc...", u, Pi)
              + np.einsum("c...,ab...->abc...", u, Pi))
        fhat = fhat + wq * np.einsum("qabc,abc...->q...", H3, a3) / (6 * CS2**3)
    cF = np.einsum("qa,a...->q...", cd, np.broadcast_to(Fv, u.shape))
    uF = (u * Fv).sum(axis=0)
    S = wq * ((cF - uF[None]) / CS2 + cu * cF / CS2**2)
    return feq + (1.0 - omega) * fhat + (1.0 - 0.5 * omega) * S


def _inside_after_shift(shape_zyx, c, bb, sign):
    """Mask over nodes x: is x + sign*c inside the domain on every wall axis?"""
    nz, ny, nx = shape_zyx
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ok = np.ones(shape_zyx, dtype=bool)
    for ax, coord, n in ((0, x, nx), (1, y, ny), (2, z, nz)):
        if bb[ax]:
            t = coord + sign * c[ax]
            ok &= (t >= 0) & (t < n)
    return ok


def _wall_gain(shape_zyx, ca, wa, bb, wall_u, rho0):
    """Population f_a(x) that returns by bounce-back comes from the link
    -c_a of x itself and gains 2 t_a rho0 (c_a . u_w)/cs2, u_w summed over the
    walls that x - c_a lies beyond (moving-wall halfway bounce-back)."""
    nz, ny, nx = shape_zyx
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cu = np.zeros(shape_zyx)
    for ax, coord, n in ((0, x, nx), (1, y, ny), (2, z, nz)):
        if not bb[ax]:
            continue
        src = coord - ca[ax]
        for side, beyond in ((0, src < 0), (1, src >= n)):
            cu += beyond * float(np.dot(ca, wall_u[ax][side]))
    return 2.0 * wa * rho0 * cu / CS2


def _stream(fpc, c, opp, bb, w=None, wall_u=None, rho0=1.0):
    """Push streaming with periodic wrap and halfway bounce-back (moving walls
    when wall_u[axis][side] is given)."""
    out = np.empty_like(fpc)
    shape = fpc.shape[1:]
    for a in range(len(c)):
        moved = np.roll(fpc[a], shift=(c[a][2], c[a][1], c[a][0]), axis=(0, 1, 2))
        has_source = _inside_after_shift(shape, c[a], bb, -1)
        back = fpc[opp[a]]
        if wall_u is not None:
            back = back + _wall_gain(shape, c[a].astype(np.float64), w[a], bb, wall_u, rho0)
        out[a] = np.where(has_source, moved, back)
    return out


def _gradient(phi, c, w, bb):
    """Isotropic gradient (1/cs2) sum_b t_b c_b phi(x + c_b); beyond a wall the
    node's own value is used."""
    G = np.zeros((3,) + phi.shape, dtype=phi.dtype)
    w = w.astype(phi.dtype)
    for b in range(len(c)):
        nb = np.roll(phi, shift=(-c[b][2], -c[b][1], -c[b][0]), axis=(0, 1, 2))
        nb = np.where(_inside_after_shift(phi.shape, c[b], bb, +1), nb, phi)
        for al in range(3):
            G[al] += w[b] * c[b][al] * nb
    return G / CS2


def _nci_force(ph, rr, G, G2, c, bb, strength, eps, reach, D):
    """Near-contact force field (Section 2.2) in gather form: node y is
    flagged when it is not bulk and, for some direction c, the node
    y - d c is bulk while y - 2 d c is not (that bulk node then sees
    interfaces on both sides along c); points beyond a wall do not count.
    Flagged nodes with a defined gradient get strength * rho_R * G/|G|."""
    thr = -1.0 + eps
    flag = np.zeros(ph.shape, dtype=bool)
    for ca in c:
        if not ca.any():
            continue
        k1 = reach * ca
        mid = np.roll(ph, shift=(k1[2], k1[1], k1[0]), axis=(0, 1, 2))
        far = np.roll(ph, shift=(2 * k1[2], 2 * k1[1], 2 * k1[0]), axis=(0, 1, 2))
        ok = (_inside_after_shift(ph.shape, ca, bb, -reach)
              & _inside_after_shift(ph.shape, ca, bb, -2 * reach))
        flag |= ok & (mid < thr) & (far > thr)
    flag &= ph > thr
    big = G2 > 1e-20
    scale = np.where(flag & big, strength * rr / np.sqrt(np.where(big, G2, 1.0)), 0.0)
    return flag, scale[None] * G[:D]


_B = {
    9: {0: -4 / 27, 1: 2 / 27, 2: 5 / 108},
    19: {0: -1 / 3, 1: 1 / 18, 2: 1 / 36},
}


def simulate(p, rho, u, nsteps, phi=None, dtype=np.float64):
    """Equilibrium start from (rho, u[, phi]), nsteps steps, then moments.

    ``p`` is an ``oracle.Params``.  Returns the same dict as
    ``oracle.moments`` (float64 arrays).  ``dtype`` np.float32 runs every
    array and constant in float32 (a plain float32 transcription of the same
    step, used to measure the step's float32 rounding floor).
    """
    c, w, opp = velocity_set(p.lattice)
    w = w.astype(dtype)
    D = p.D
    shape = (p.nz, p.ny, p.nx)
    Q = len(w)
    rho = np.asarray(rho, dtype=dtype).reshape(shape)
    u = np.asarray(u, dtype=dtype).reshape((D,) + shape)
    F = tuple(p.force)
    cd = c[:, :D].astype(dtype)
    wq = w.reshape(Q, 1, 1, 1)

    def feq_of(r, uv):
        cu = np.einsum("qa,a...->q...", cd, uv)
        usq = (uv * uv).sum(axis=0)
        e = cu / CS2 + 0.5 * (cu / CS2) ** 2 - 0.5 * usq / CS2
        out = wq * (r[None] + p.rho0 * e)
        if p.order >= 3:
            _, _, H3 = _hermite(c, D, dtype)
            uuu = np.einsum("a...,b...,c...->abc...", uv, uv, uv)
            out = out + wq * p.rho0 * np.einsum("qabc,abc...->q...", H3, uuu) / (6 * CS2**3)
        return out

    wu = None if p.wall_u is None else np.asarray(p.wall_u, dtype=np.float64).reshape(3, 2, 3)
    f0 = feq_of(rho, u)
    if p.species == 1:
        f = f0
        for _ in range(nsteps):
            f = _stream(_collide(f, c, w, D, p.tau, p.rho0, F, p.order), c, opp, p.bb, w, wu,
                        p.rho0)
        g = f
        ph = None
    else:
        phi = np.asarray(phi, dtype=dtype).reshape(shape)
        fr = 0.5 * (1 + phi)[None] * f0
        fb = 0.5 * (1 - phi)[None] * f0
        Bv = np.array([_B[p.lattice][int((ci * ci).sum())] for ci in c],
                      dtype=dtype).reshape(Q, 1, 1, 1)
        norm_c = np.sqrt((c * c).sum(axis=1)).astype(dtype)
        omega = 1.0 / p.tau
        for _ in range(nsteps):
            rr, rb = fr.sum(axis=0), fb.sum(axis=0)
            r = rr + rb
            ph = (rr - rb) / r
            G = _gradient(ph, c, w, p.bb)
            G2 = (G * G).sum(axis=0)
            Gn = np.sqrt(G2)
            Fs = F
            if p.nci_strength != 0.0:
                _, Fn = _nci_force(ph, rr, G, G2, c, p.bb, p.nci_strength, p.nci_eps,
                                   p.nci_reach, D)
                Fs = np.asarray(F[:D], dtype=dtype).reshape((D, 1, 1, 1)) + Fn
            gpc = _collide(fr + fb, c, w, D, p.tau, p.rho0, Fs, p.order)
            cG = np.einsum("qa,a...->q...", c.astype(dtype), G)
            big = (G2 > 1e-20)[None]
            safe = np.where(big, G2[None], 1.0)
            pert = np.where(big, 2.25 * p.sigma * omega * Gn[None] * (wq * cG * cG / safe - Bv), 0.0)
            nc = norm_c.reshape(Q, 1, 1, 1)
            cosang = np.where(big & (nc > 0), cG / np.where(nc > 0, nc, 1.0) / np.sqrt(safe), 0.0)
            gs = gpc + pert
            rec = p.beta * (rr * rb / r)[None] * wq * cosang
            fr = _stream((rr / r)[None] * gs + rec, c, opp, p.bb)
            fb = _stream((rb / r)[None] * gs - rec, c, opp, p.bb)
        g = fr + fb
        rr, rb = fr.sum(axis=0), fb.sum(axis=0)
        ph = (rr - rb) / (rr + rb)
        masses = (float(fr.sum(dtype=np.float64)), float(fb.sum(dtype=np.float64)))

    r = g.sum(axis=0)
    j = np.einsum("qa,q...->a...", cd, g)
    Fv = np.asarray(F[:D], dtype=dtype).reshape((D, 1, 1, 1))
    uo = (j + 0.5 * Fv) / p.rho0
    fe = feq_of(r, uo)
    Pi = np.einsum("qa,qb,q...->ab...", cd, cd, g - fe)
    if D == 2:
        pineq = np.stack([Pi[0, 0], Pi[1, 1], Pi[0, 1]])
    else:
        pineq = np.stack([Pi[0, 0], Pi[1, 1], Pi[2, 2], Pi[0, 1], Pi[0, 2], Pi[1, 2]])
    N = p.N
    f64 = np.float64
    out = {"rho": r.reshape(N).astype(f64), "u": uo.reshape(D, N).astype(f64),
           "pineq": pineq.reshape(-1, N).astype(f64)}
    if ph is not None:
        out["phi"] = ph.reshape(N).astype(f64)
        out["mass_red"], out["mass_blue"] = masses
    return out
