"""Independent numpy membership tests for the solid families (test helper).

These restate solid membership with a different formulation from the oracle
(angles via atan2, radii interpolated end to end) so that the oracle's
signed-distance components, normals and ray distances can be checked against
plain geometry.  Each function returns (inside, margin) where margin is a
lower estimate of the distance to the nearest face, used to keep test points
away from surfaces.
"""
import math

import numpy as np

BOX, TUBS, CONS, ORB, TRD, SPHERE = 0, 1, 2, 3, 4, 5


def _phi_member(p, sphi, dphi):
    if dphi >= 2 * math.pi:
        return np.ones(len(p), bool), np.full(len(p), np.inf)
    ang = np.mod(np.arctan2(p[:, 1], p[:, 0]) - sphi, 2 * math.pi)
    inside = ang < dphi
    rho = np.hypot(p[:, 0], p[:, 1])
    # angular distance to the nearer plane, times the radius (planes are half-planes)
    da = np.minimum(np.abs(ang), np.abs(ang - dphi))
    da = np.minimum(da, np.abs(2 * math.pi - ang))
    margin = rho * np.sin(np.minimum(da, math.pi / 2))
    return inside, margin


def member(stype, par, p):
    p = np.atleast_2d(np.asarray(p, dtype=np.float64))
    if stype == BOX:
        h = np.asarray(par[:3])
        q = np.abs(p) - h
        return np.all(q < 0, axis=1), np.min(np.abs(q), axis=1)
    if stype == ORB:
        r = np.linalg.norm(p, axis=1)
        return r < par[0], np.abs(r - par[0])
    if stype == SPHERE:
        # spherical coordinates: r, polar angle from +z, azimuth
        rmin, rmax, sphi, dphi, st, dt = par[:6]
        r = np.linalg.norm(p, axis=1)
        th = np.arccos(np.clip(p[:, 2] / np.maximum(r, 1e-300), -1.0, 1.0))
        inr = (r < rmax) & ((r > rmin) | (rmin == 0))
        lo_ok = (th > st) | (st == 0)
        hi_ok = (th < st + dt) | (st + dt >= math.pi)
        inphi, mphi = _phi_member(p, sphi, dphi)
        m = np.abs(r - rmax)
        if rmin > 0:
            m = np.minimum(m, np.abs(r - rmin))
        for tb, on in ((st, st > 0), (st + dt, st + dt < math.pi)):
            if on:
                m = np.minimum(m, r * np.abs(np.sin(np.minimum(np.abs(th - tb), math.pi / 2))))
        m = np.minimum(m, mphi)
        return inr & lo_ok & hi_ok & inphi, m
    if stype == TRD:
        # half widths interpolated end to end between z = -dz and z = +dz
        dx1, dx2, dy1, dy2, dz = par[:5]
        z = p[:, 2]
        f = (z + dz) / (2 * dz)
        hx = dx1 + (dx2 - dx1) * f
        hy = dy1 + (dy2 - dy1) * f
        inside = (np.abs(z) < dz) & (np.abs(p[:, 0]) < hx) & (np.abs(p[:, 1]) < hy)
        tx = math.atan2(dx2 - dx1, 2 * dz)
        ty = math.atan2(dy2 - dy1, 2 * dz)
        m = np.minimum(np.abs(np.abs(z) - dz), np.abs(hx - np.abs(p[:, 0])) * math.cos(tx))
        m = np.minimum(m, np.abs(hy - np.abs(p[:, 1])) * math.cos(ty))
        return inside, m
    if stype == TUBS:
        rmin1 = rmin2 = par[0]
        rmax1 = rmax2 = par[1]
        dz, sphi, dphi = par[2], par[3], par[4]
    else:
        rmin1, rmax1, rmin2, rmax2, dz, sphi, dphi = par[:7]
    z = p[:, 2]
    f = (z + dz) / (2 * dz)
    rmin = rmin1 + (rmin2 - rmin1) * f
    rmax = rmax1 + (rmax2 - rmax1) * f
    rho = np.hypot(p[:, 0], p[:, 1])
    inz = np.abs(z) < dz
    inr = (rho < rmax) & ((rho > rmin) | ((rmin1 == 0) & (rmin2 == 0)))
    inphi, mphi = _phi_member(p, sphi, dphi)
    slope_o = (rmax2 - rmax1) / (2 * dz)
    slope_i = (rmin2 - rmin1) / (2 * dz)
    m = np.minimum(np.abs(np.abs(z) - dz), np.abs(rho - rmax) / math.sqrt(1 + slope_o ** 2))
    if rmin1 > 0 or rmin2 > 0:
        m = np.minimum(m, np.abs(rho - rmin) / math.sqrt(1 + slope_i ** 2))
    m = np.minimum(m, mphi)
    return inz & inr & inphi, m


def compose_touchables(desc, parent, pv):
    """Global (R, t) of every touchable: x_global = R x_local + t."""
    n = len(parent)
    Rg = np.zeros((n, 3, 3))
    tg = np.zeros((n, 3))
    Rg[0] = np.eye(3)
    for i in range(1, n):
        P = parent[i]
        R = desc.pv_rot[pv[i]].reshape(3, 3)
        t = desc.pv_trans[pv[i]]
        Rg[i] = Rg[P] @ R
        tg[i] = Rg[P] @ t + tg[P]
    return Rg, tg


def locate_bruteforce(desc, parent, pv, lv, depth, pts):
    """Deepest touchable containing each point, testing every touchable."""
    Rg, tg = compose_touchables(desc, parent, pv)
    n = len(parent)
    best = np.full(len(pts), -1)
    bestd = np.full(len(pts), -1)
    margin = np.full(len(pts), np.inf)
    for i in range(n):
        loc = (pts - tg[i]) @ Rg[i]
        s = desc.lv_solid[lv[i]]
        ins, m = member(desc.solid_type[s], desc.solid_par[s], loc)
        margin = np.minimum(margin, m)
        upd = ins & (depth[i] > bestd)
        best[upd] = i
        bestd[upd] = depth[i]
    return best, margin
