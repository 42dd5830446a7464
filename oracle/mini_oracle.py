"""Independent vectorised NumPy FP64 implementation of the same SALE step
(test infrastructure, small meshes only).

It is written separately from ``sale_oracle.c`` -- whole-array slicing with
zero padding instead of per-element loops, and a 3-point Gauss-Legendre rule
for the swept volumes instead of the 2-point one -- so that an indexing,
sign or boundary mistake in either implementation shows up as a
disagreement. The steps follow the same fixed reading O1..O12 of the
ScalSALE SALE step (Lagrangian phase, Eulerian rezone and advection;
Sec. I-D and Table I of the paper).

Arrays: cells (nz, ny, nx), nodes (nz+1, ny+1, nx+1), x fastest.
"""
import numpy as np

_G3 = np.array([0.5 - 0.5 * np.sqrt(0.6), 0.5, 0.5 + 0.5 * np.sqrt(0.6)])
_W3 = np.array([5.0, 8.0, 5.0]) / 18.0


def swept_volume(d00, d10, d01, d11, h1, h2):
    """Exact swept volume of faces with bilinear displacement (vectorised).
    d.. are (..., 3) with components (normal, t1, t2); corners (s,t)."""
    vol = 0.0
    for a in range(3):
        for b in range(3):
            s, t = _G3[a], _G3[b]
            d = d00 * (1 - s) * (1 - t) + d10 * s * (1 - t) + d01 * (1 - s) * t + d11 * s * t
            ds = (d10 - d00) * (1 - t) + (d11 - d01) * t
            dt = (d01 - d00) * (1 - s) + (d11 - d10) * s
            xi, eta, zeta = d[..., 0], d[..., 1], d[..., 2]
            trip = np.einsum("...i,...i->...", d, np.cross(ds, dt))
            f = (h1 * h2 * xi + 0.5 * h1 * (xi * dt[..., 2] - zeta * dt[..., 0])
                 + 0.5 * h2 * (xi * ds[..., 1] - eta * ds[..., 0]) + trip / 3.0)
            vol = vol + _W3[a] * _W3[b] * f
    return vol


def _pad(a):
    return np.pad(a, 1)


def _cells_to_nodes_sum(cf):
    """sum over the (up to 8) existing cells around every node."""
    p = _pad(cf)
    return (p[:-1, :-1, :-1] + p[:-1, :-1, 1:] + p[:-1, 1:, :-1] + p[:-1, 1:, 1:]
            + p[1:, :-1, :-1] + p[1:, :-1, 1:] + p[1:, 1:, :-1] + p[1:, 1:, 1:])


def _nodes_to_cells_sum(nf):
    return (nf[:-1, :-1, :-1] + nf[:-1, :-1, 1:] + nf[:-1, 1:, :-1] + nf[:-1, 1:, 1:]
            + nf[1:, :-1, :-1] + nf[1:, :-1, 1:] + nf[1:, 1:, :-1] + nf[1:, 1:, 1:])


def _nodes_to_cells_max(nf):
    return np.maximum.reduce([nf[:-1, :-1, :-1], nf[:-1, :-1, 1:], nf[:-1, 1:, :-1], nf[:-1, 1:, 1:],
                              nf[1:, :-1, :-1], nf[1:, :-1, 1:], nf[1:, 1:, :-1], nf[1:, 1:, 1:]])


def _corner_dot(X, Y, Z, dx, dy, dz):
    """sum_p S_{c,p} . (X,Y,Z)_p for every cell."""
    ddx = X[:, :, 1:] - X[:, :, :-1]
    ddy = Y[:, 1:, :] - Y[:, :-1, :]
    ddz = Z[1:, :, :] - Z[:-1, :, :]
    sx = ddx[:-1, :-1, :] + ddx[:-1, 1:, :] + ddx[1:, :-1, :] + ddx[1:, 1:, :]
    sy = ddy[:-1, :, :-1] + ddy[:-1, :, 1:] + ddy[1:, :, :-1] + ddy[1:, :, 1:]
    sz = ddz[:, :-1, :-1] + ddz[:, :-1, 1:] + ddz[:, 1:, :-1] + ddz[:, 1:, 1:]
    return dy * dz / 4 * sx + dz * dx / 4 * sy + dx * dy / 4 * sz


def _vanleer(am, ap):
    """harmonic slope limiter, zero unless the one-sided slopes share a sign"""
    prod = am * ap
    den = np.where(prod > 0, am + ap, 1.0)
    return np.where(prod > 0, 2.0 * prod / den, 0.0)


def _limited_slopes(q, ax, h):
    """limited slope of q along array axis ax; zero at the first and last
    entry along that axis (a wall on that side)"""
    d = np.diff(q, axis=ax) / h
    out = np.zeros_like(q)
    n = q.shape[ax]
    if n >= 3:
        mid = [slice(None)] * 3
        mid[ax] = slice(1, n - 1)
        a = [slice(None)] * 3
        a[ax] = slice(0, n - 2)
        b = [slice(None)] * 3
        b[ax] = slice(1, n - 1)
        out[tuple(mid)] = _vanleer(d[tuple(a)], d[tuple(b)])
    return out


def _face_value(q_lo, s_lo, q_hi, s_hi, dv, area, h):
    """second-order donor value of faces with swept volume dv between the
    lower and upper neighbours: the limited linear profile of the donor at
    the centroid of the swept slab"""
    off = 0.5 * (h - np.abs(dv) / area)
    return np.where(dv > 0, q_lo + s_lo * off, q_hi - s_hi * off)


def _zero_walls(u, v, w):
    u[:, :, 0] = 0.0
    u[:, :, -1] = 0.0
    v[:, 0, :] = 0.0
    v[:, -1, :] = 0.0
    w[0, :, :] = 0.0
    w[-1, :, :] = 0.0


def step(grid, rho, e, u, v, w, t):
    """One step. Returns (rho, e, u, v, w, t_new, dt) as new arrays."""
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    dx, dy, dz = grid.spacing
    V0 = dx * dy * dz
    h = min(dx, dy, dz)
    gm = grid.gamma
    m = rho * V0
    p = (gm - 1) * rho * e
    c = np.sqrt(gm * (gm - 1) * np.maximum(e, 0.0))
    D = _corner_dot(u, v, w, dx, dy, dz) / V0
    q = np.where(D < 0, rho * (grid.cq * (h * D) ** 2 + grid.cl * c * h * np.abs(D)), 0.0)
    spd = _nodes_to_cells_max(np.sqrt(u * u + v * v + w * w))
    a = c + spd + 4 * grid.cq * h * np.maximum(-D, 0.0)
    amax = a.max()
    dt = grid.cfl * h / amax if amax > 0 else grid.t_end - t
    dt = min(dt, grid.t_end - t)
    # predictor
    dVs = 0.5 * dt * V0 * D
    rs = m / (V0 + dVs)
    es = e - (p + q) * dVs / m
    Ps = (gm - 1) * rs * es + q
    # nodal mass and forces
    mp = 0.125 * _cells_to_nodes_sum(m)
    Pp = _pad(Ps)
    Fx = sum(Pp[1 - t2:2 - t2 + nz, 1 - t1:2 - t1 + ny, 0:nx + 1]
             - Pp[1 - t2:2 - t2 + nz, 1 - t1:2 - t1 + ny, 1:nx + 2] for t1 in (0, 1) for t2 in (0, 1))
    Fy = sum(Pp[1 - t2:2 - t2 + nz, 0:ny + 1, 1 - t1:2 - t1 + nx]
             - Pp[1 - t2:2 - t2 + nz, 1:ny + 2, 1 - t1:2 - t1 + nx] for t1 in (0, 1) for t2 in (0, 1))
    Fz = sum(Pp[0:nz + 1, 1 - t2:2 - t2 + ny, 1 - t1:2 - t1 + nx]
             - Pp[1:nz + 2, 1 - t2:2 - t2 + ny, 1 - t1:2 - t1 + nx] for t1 in (0, 1) for t2 in (0, 1))
    u1 = u + dt * (dy * dz / 4 * Fx) / mp
    v1 = v + dt * (dz * dx / 4 * Fy) / mp
    w1 = w + dt * (dx * dy / 4 * Fz) / mp
    _zero_walls(u1, v1, w1)
    ub, vb, wb = 0.5 * (u + u1), 0.5 * (v + v1), 0.5 * (w + w1)
    eL = e - dt / m * Ps * _corner_dot(ub, vb, wb, dx, dy, dz)
    # swept volumes
    dlt = np.stack([dt * ub, dt * vb, dt * wb], axis=-1)  # (nz+1, ny+1, nx+1, 3)
    dvx = np.zeros((nz, ny, nx + 1))
    dvy = np.zeros((nz, ny + 1, nx))
    dvz = np.zeros((nz + 1, ny, nx))
    if nx > 1:
        dd = dlt[:, :, 1:nx][..., [0, 1, 2]]
        dvx[:, :, 1:nx] = swept_volume(dd[:-1, :-1], dd[:-1, 1:], dd[1:, :-1], dd[1:, 1:], dy, dz)
    if ny > 1:
        dd = dlt[:, 1:ny, :][..., [1, 2, 0]]
        dvy[:, 1:ny, :] = swept_volume(dd[:-1, :, :-1], dd[1:, :, :-1], dd[:-1, :, 1:], dd[1:, :, 1:], dz, dx)
    if nz > 1:
        dd = dlt[1:nz, :, :][..., [2, 0, 1]]
        dvz[1:nz, :, :] = swept_volume(dd[:, :-1, :-1], dd[:, :-1, 1:], dd[:, 1:, :-1], dd[:, 1:, 1:], dx, dy)
    VL = V0 + (dvx[:, :, 1:] - dvx[:, :, :-1]) + (dvy[:, 1:, :] - dvy[:, :-1, :]) + (dvz[1:] - dvz[:-1])
    if np.any(VL <= 0):
        raise FloatingPointError("tangled cell")
    rhoL = m / VL
    # donor-cell face fluxes (order 2: donor values from limited linear profiles)
    o2 = getattr(grid, "order", 1) == 2
    mux = np.zeros_like(dvx)
    exf = np.zeros_like(dvx)
    f = dvx[:, :, 1:nx]
    if o2:
        sr, se = _limited_slopes(rhoL, 2, dx), _limited_slopes(eL, 2, dx)
        dr = _face_value(rhoL[:, :, :-1], sr[:, :, :-1], rhoL[:, :, 1:], sr[:, :, 1:], f, dy * dz, dx)
        de = _face_value(eL[:, :, :-1], se[:, :, :-1], eL[:, :, 1:], se[:, :, 1:], f, dy * dz, dx)
    else:
        dr = np.where(f > 0, rhoL[:, :, :-1], rhoL[:, :, 1:])
        de = np.where(f > 0, eL[:, :, :-1], eL[:, :, 1:])
    mux[:, :, 1:nx] = dr * f
    exf[:, :, 1:nx] = dr * f * de
    muy = np.zeros_like(dvy)
    eyf = np.zeros_like(dvy)
    f = dvy[:, 1:ny, :]
    if o2:
        sr, se = _limited_slopes(rhoL, 1, dy), _limited_slopes(eL, 1, dy)
        dr = _face_value(rhoL[:, :-1, :], sr[:, :-1, :], rhoL[:, 1:, :], sr[:, 1:, :], f, dz * dx, dy)
        de = _face_value(eL[:, :-1, :], se[:, :-1, :], eL[:, 1:, :], se[:, 1:, :], f, dz * dx, dy)
    else:
        dr = np.where(f > 0, rhoL[:, :-1, :], rhoL[:, 1:, :])
        de = np.where(f > 0, eL[:, :-1, :], eL[:, 1:, :])
    muy[:, 1:ny, :] = dr * f
    eyf[:, 1:ny, :] = dr * f * de
    muz = np.zeros_like(dvz)
    ezf = np.zeros_like(dvz)
    f = dvz[1:nz]
    if o2:
        sr, se = _limited_slopes(rhoL, 0, dz), _limited_slopes(eL, 0, dz)
        dr = _face_value(rhoL[:-1], sr[:-1], rhoL[1:], sr[1:], f, dx * dy, dz)
        de = _face_value(eL[:-1], se[:-1], eL[1:], se[1:], f, dx * dy, dz)
    else:
        dr = np.where(f > 0, rhoL[:-1], rhoL[1:])
        de = np.where(f > 0, eL[:-1], eL[1:])
    muz[1:nz] = dr * f
    ezf[1:nz] = dr * f * de
    netm = (mux[:, :, 1:] - mux[:, :, :-1]) + (muy[:, 1:, :] - muy[:, :-1, :]) + (muz[1:] - muz[:-1])
    nete = (exf[:, :, 1:] - exf[:, :, :-1]) + (eyf[:, 1:, :] - eyf[:, :-1, :]) + (ezf[1:] - ezf[:-1])
    M = m - netm
    rn = rho - netm / V0
    epre = eL + (eL * netm - nete) / M
    # dual-mesh fluxes: phi on node edges
    sxc = np.pad(mux[:, :, :-1] + mux[:, :, 1:], ((1, 1), (1, 1), (0, 0)))
    phx = 0.125 * (sxc[:-1, :-1] + sxc[:-1, 1:] + sxc[1:, :-1] + sxc[1:, 1:])  # (nz+1, ny+1, nx)
    syc = np.pad(muy[:, :-1, :] + muy[:, 1:, :], ((1, 1), (0, 0), (1, 1)))
    phy = 0.125 * (syc[:-1, :, :-1] + syc[:-1, :, 1:] + syc[1:, :, :-1] + syc[1:, :, 1:])  # (nz+1, ny, nx+1)
    szc = np.pad(muz[:-1] + muz[1:], ((0, 0), (1, 1), (1, 1)))
    phz = 0.125 * (szc[:, :-1, :-1] + szc[:, :-1, 1:] + szc[:, 1:, :-1] + szc[:, 1:, 1:])  # (nz, ny+1, nx+1)
    # dual swept volumes on node edges, averaged like the dual mass fluxes
    sxv = np.pad(dvx[:, :, :-1] + dvx[:, :, 1:], ((1, 1), (1, 1), (0, 0)))
    dvpx = 0.125 * (sxv[:-1, :-1] + sxv[:-1, 1:] + sxv[1:, :-1] + sxv[1:, 1:])
    syv = np.pad(dvy[:, :-1, :] + dvy[:, 1:, :], ((1, 1), (0, 0), (1, 1)))
    dvpy = 0.125 * (syv[:-1, :, :-1] + syv[:-1, :, 1:] + syv[1:, :, :-1] + syv[1:, :, 1:])
    szv = np.pad(dvz[:-1] + dvz[1:], ((0, 0), (1, 1), (1, 1)))
    dvpz = 0.125 * (szv[:, :-1, :-1] + szv[:, :-1, 1:] + szv[:, 1:, :-1] + szv[:, 1:, 1:])
    vel = np.stack([u1, v1, w1], axis=-1)
    Pm = mp[..., None] * vel
    K = 0.5 * mp * (u1 * u1 + v1 * v1 + w1 * w1)
    for axis, ph, dvp, hh, area in ((2, phx, dvpx, dx, dy * dz), (1, phy, dvpy, dy, dz * dx),
                                    (0, phz, dvpz, dz, dx * dy)):
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        if o2:
            # the donor's swept slab lies on the flux's side: sign from phi
            sdv = np.where(ph > 0, np.abs(dvp), -np.abs(dvp))
            ud = np.stack([_face_value(vel[..., m][lo], _limited_slopes(vel[..., m], axis, hh)[lo],
                                       vel[..., m][hi], _limited_slopes(vel[..., m], axis, hh)[hi],
                                       sdv, area, hh) for m in range(3)], axis=-1)
        else:
            ud = np.where((ph > 0)[..., None], vel[lo], vel[hi])
        Pi = ph[..., None] * ud
        ka = ph * 0.5 * np.sum(ud * ud, axis=-1)
        Pm[lo] -= Pi
        Pm[hi] += Pi
        K[lo] -= ka
        K[hi] += ka
    mn = 0.125 * _cells_to_nodes_sum(M)
    un, vn, wn = Pm[..., 0] / mn, Pm[..., 1] / mn, Pm[..., 2] / mn
    _zero_walls(un, vn, wn)
    dK = K - 0.5 * mn * (un * un + vn * vn + wn * wn)
    en = epre + 0.125 * _nodes_to_cells_sum(dK / mn)
    return rn, en, un, vn, wn, t + dt, dt
