"""ctypes wrapper of the plain C oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg use this package.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gnav_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# Counter slots, fate and limiter codes (same values as in the C source).
COUNTERS = ["steps", "pe", "compton", "pair", "crossings", "escaped", "cutoff", "pushes",
            "stuck", "truncated", "tracks"]
LIM_MOTHER, LIM_PE, LIM_COMPTON, LIM_PAIR = -1, -2, -3, -4
FATE_ABSORBED, FATE_ESCAPED, FATE_CUTOFF, FATE_STUCK, FATE_TRUNCATED, FATE_PAIR = 1, 2, 3, 4, 5, 6
ME = 0.51099895

LOG_DTYPE = np.dtype([("touchable", np.int32), ("code", np.int32), ("step", np.float64),
                      ("edep", np.float64), ("energy", np.float64)])
DIGEST_DTYPE = np.dtype([("hash", np.uint64), ("n", np.int32), ("fate", np.int32),
                         ("sum_step", np.float64), ("sum_edep", np.float64)])


def build(force=False):
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        L.og_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.og_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.og_uniform.restype = C.c_double
        L.og_kn_per_electron.argtypes = [C.c_longdouble]
        L.og_kn_per_electron.restype = C.c_longdouble
        L.og_sigma_atom.argtypes = [C.c_int, C.c_double, f64p]
        L.og_create.restype = P
        L.og_create.argtypes = [C.c_int, i32p, f64p, C.c_int, f64p, i32p, i32p, f64p, f64p,
                                C.c_int, i32p, i32p, i32p, i32p, C.c_int, i32p, f64p, f64p, C.c_int]
        L.og_destroy.argtypes = [P]
        L.og_n_touchables.argtypes = [P]
        L.og_n_touchables.restype = C.c_int
        L.og_touchables.argtypes = [P, i32p, i32p, i32p, i32p]
        L.og_set_paper_mode.argtypes = [P, C.c_int, C.c_double]
        L.og_set_voxels.argtypes = [P, C.c_int]
        L.og_set_voxels.restype = C.c_int
        L.og_mu.argtypes = [P, C.c_int, C.c_int, f64p, f64p]
        L.og_table.argtypes = [P, f64p, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.og_locate.argtypes = [P, C.c_int, f64p, P, i32p]
        L.og_compute_step.argtypes = [P, C.c_int, f64p, f64p, P, f64p, i32p, P]
        L.og_compute_safety.argtypes = [P, C.c_int, f64p, P, f64p]
        L.og_compute_step_normal.argtypes = [P, C.c_int, f64p, f64p, P, f64p, i32p, P, f64p, i32p]
        L.og_solid_normal_n.argtypes = [C.c_int, f64p, C.c_int, f64p, f64p, i32p]
        L.og_solid_normal_n.restype = C.c_int
        L.og_solid_eval.argtypes = [C.c_int, f64p, C.c_int, C.c_int, f64p, P, f64p]
        L.og_solid_eval.restype = C.c_int
        L.og_free_path.argtypes = [P, f64p, f64p, C.c_double, C.c_double, C.POINTER(C.c_int)]
        L.og_free_path.restype = C.c_double
        L.og_compton_sample_n.argtypes = [C.c_double, C.c_int, C.c_uint64, f64p, f64p, i32p]
        L.og_rotate.argtypes = [C.c_int, f64p, f64p, f64p]
        L.og_transport.argtypes = [P, C.c_int64, i32p, i32p, f64p, f64p, f64p, C.c_uint64,
                                   C.c_double, C.c_int64, f64p, f64p, f64p, u64p, P, C.c_int64,
                                   P, P, P, P, P, P]
        L.og_transport.restype = C.c_int
        _lib = L
    return _lib


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    lib().og_philox4x32_10(_c(ctr, np.uint32), _c(key, np.uint32), out)
    return out


def uniform(seed, event, key, draw):
    return lib().og_uniform(seed, event, key, draw)


def sigma_atom(Z, E):
    out = np.zeros(3)
    lib().og_sigma_atom(int(Z), float(E), out)
    return out


def kn_per_electron(k):
    return float(lib().og_kn_per_electron(k))


SOLID_OPS = {"d": 0, "inside": 1, "dist_in": 2, "dist_out": 3, "safety_in": 4, "safety_out": 5}


def solid_eval(stype, par, op, p, v=None):
    par8 = np.zeros(8)
    par8[: len(par)] = par
    p = _c(np.atleast_2d(p), np.float64)
    n = p.shape[0]
    vv = None if v is None else _c(np.broadcast_to(np.atleast_2d(v), (n, 3)), np.float64)
    out = np.zeros(n)
    rc = lib().og_solid_eval(int(stype), par8, SOLID_OPS[op], n, p, _ptr(vv), out)
    if rc != 0:
        raise ValueError("invalid solid parameters")
    return out


def solid_normal(stype, par, p):
    """Outward unit normals of a solid at points p [n][3] and the number of faces
    within the tolerance of the defining one (1 face, 2+ edge or corner)."""
    par8 = np.zeros(8)
    par8[: len(par)] = par
    p = _c(np.atleast_2d(p), np.float64)
    out = np.zeros_like(p)
    faces = np.zeros(p.shape[0], np.int32)
    if lib().og_solid_normal_n(int(stype), par8, p.shape[0], p, out, faces) != 0:
        raise ValueError("invalid solid parameters")
    return out, faces


def compton_sample(E, n, seed=0):
    eps = np.zeros(n)
    cost = np.zeros(n)
    draws = np.zeros(n, dtype=np.int32)
    lib().og_compton_sample_n(float(E), int(n), int(seed), eps, cost, draws)
    return eps, cost, draws


def rotate(v, cost, phi):
    v = _c(v, np.float64).copy()
    lib().og_rotate(v.shape[0], v, _c(cost, np.float64), _c(phi, np.float64))
    return v


class Geometry:
    """The oracle's own view of a flat geometry description."""

    def __init__(self, desc):
        L = lib()
        self.desc = desc
        self._keep = [
            _c(desc.solid_type, np.int32), _c(desc.solid_par, np.float64),
            _c(desc.mat_density, np.float64), _c(desc.mat_el_off, np.int32),
            _c(desc.el_Z, np.int32) if desc.el_Z.size else np.zeros(1, np.int32),
            _c(desc.el_A, np.float64) if desc.el_A.size else np.zeros(1),
            _c(desc.el_wfrac, np.float64) if desc.el_wfrac.size else np.zeros(1),
            _c(desc.lv_solid, np.int32), _c(desc.lv_mat, np.int32), _c(desc.lv_dau_off, np.int32),
            _c(desc.lv_dau_cnt, np.int32),
            _c(desc.pv_lv, np.int32) if desc.n_pv else np.zeros(1, np.int32),
            _c(desc.pv_rot, np.float64) if desc.n_pv else np.zeros(9),
            _c(desc.pv_trans, np.float64) if desc.n_pv else np.zeros(3),
        ]
        k = self._keep
        h = L.og_create(desc.n_solids, k[0], k[1], desc.n_mats, k[2], k[3], k[4], k[5], k[6],
                        desc.n_lv, k[7], k[8], k[9], k[10], desc.n_pv, k[11], k[12], k[13],
                        int(desc.world_lv))
        if not h:
            raise ValueError(f"oracle rejected geometry {desc.name}")
        self.h = h
        self.n_touchables = L.og_n_touchables(h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().og_destroy(h)
            self.h = None

    def touchables(self):
        n = self.n_touchables
        parent, pv, lv, depth = (np.zeros(n, np.int32) for _ in range(4))
        lib().og_touchables(self.h, parent, pv, lv, depth)
        return parent, pv, lv, depth

    def set_paper_mode(self, on=True, mu_mass=0.06146):
        lib().og_set_paper_mode(self.h, int(on), float(mu_mass))

    def set_voxels(self, on=True):
        """Search daughters through per-mother cell grids (the oracle's faster
        CPU method; the answers equal the brute-force ones)."""
        if lib().og_set_voxels(self.h, int(on)) != 0:
            raise MemoryError("oracle voxel grids too large")

    def mu(self, mat, E):
        E = _c(np.atleast_1d(E), np.float64)
        out = np.zeros((E.shape[0], 3))
        lib().og_mu(self.h, int(mat), E.shape[0], E, out)
        return out

    def table(self):
        out = np.zeros((self.desc.n_mats, 3, 257))
        a, b = C.c_double(), C.c_double()
        lib().og_table(self.h, out, C.byref(a), C.byref(b))
        return out, a.value, b.value

    def locate(self, pos, dirs=None):
        pos = _c(pos, np.float64)
        n = pos.shape[0]
        d = None if dirs is None else _c(dirs, np.float64)
        out = np.zeros(n, np.int32)
        lib().og_locate(self.h, n, pos, _ptr(d), out)
        return out

    def compute_step(self, pos, dirs, touchable=None, with_next=True):
        pos = _c(pos, np.float64)
        dirs = _c(dirs, np.float64)
        n = pos.shape[0]
        t = None if touchable is None else _c(touchable, np.int32)
        step = np.zeros(n)
        lim = np.zeros(n, np.int32)
        nxt = np.zeros(n, np.int32) if with_next else None
        lib().og_compute_step(self.h, n, pos, dirs, _ptr(t), step, lim, _ptr(nxt))
        return step, lim, nxt

    def compute_step_normal(self, pos, dirs, touchable=None):
        """ComputeStep plus the exit normal of the crossed boundary (global frame) and its
        validity (0 none, 1 face, 2 edge or corner)."""
        pos = _c(pos, np.float64)
        dirs = _c(dirs, np.float64)
        n = pos.shape[0]
        t = None if touchable is None else _c(touchable, np.int32)
        step = np.zeros(n)
        lim = np.zeros(n, np.int32)
        nxt = np.zeros(n, np.int32)
        nrm = np.zeros((n, 3))
        val = np.zeros(n, np.int32)
        lib().og_compute_step_normal(self.h, n, pos, dirs, _ptr(t), step, lim, nxt.ctypes.data_as(C.c_void_p),
                                     nrm, val)
        return step, lim, nxt, nrm, val

    def compute_safety(self, pos, touchable=None):
        pos = _c(pos, np.float64)
        n = pos.shape[0]
        t = None if touchable is None else _c(touchable, np.int32)
        out = np.zeros(n)
        lib().og_compute_safety(self.h, n, pos, _ptr(t), out)
        return out

    def free_path(self, x0, w, E, Y):
        nb = C.c_int()
        T = lib().og_free_path(self.h, _c(x0, np.float64), _c(w, np.float64), float(E),
                               float(Y), C.byref(nb))
        return T, nb.value

    def transport(self, prim, seed=0, ecut=1e-3, max_steps=1_000_000, log_cap=0, n_events=None,
                  want_start=False, want_digest=False, want_margins=False):
        """Run the gamma loop; returns a dict of tallies, counters and optional logs (and,
        with want_start, the start state [3 n][7] = position, direction, energy of every
        track slot: 3 i the primary, 3 i + 1 and 3 i + 2 its annihilation photons); with
        want_digest the per-track digests [3 n]; with want_margins (needs log_cap) the
        smallest decision margin behind each log record [3 n][log_cap] and after the last
        record [3 n] (|a - b| / scale of the closest comparison)."""
        n = prim.n
        ne = prim.n_events if n_events is None else n_events
        edep_t = np.zeros(self.n_touchables)
        edep_ev = np.zeros(ne)
        esc_ev = np.zeros(ne)
        counters = np.zeros(len(COUNTERS), np.uint64)
        log = logn = fate = None
        if log_cap > 0:
            log = np.zeros((3 * n, log_cap), dtype=LOG_DTYPE)
            logn = np.zeros(3 * n, np.int32)
            fate = np.zeros(3 * n, np.int32)
        start = np.full((3 * n, 7), np.nan) if want_start else None
        digest = np.zeros(3 * n, DIGEST_DTYPE) if want_digest else None
        margin = np.full((3 * n, max(log_cap, 1)), np.inf, np.float32) if want_margins else None
        tail = np.full(3 * n, np.inf, np.float32) if want_margins else None
        lib().og_transport(self.h, n, _c(prim.event, np.int32), _c(prim.prim_id, np.int32),
                           _c(prim.pos, np.float64), _c(prim.dir, np.float64),
                           _c(prim.energy, np.float64), int(seed), float(ecut), int(max_steps),
                           edep_t, edep_ev, esc_ev, counters, _ptr(log), int(log_cap), _ptr(logn),
                           _ptr(fate), _ptr(start), _ptr(digest), _ptr(margin), _ptr(tail))
        out = dict(edep_touchable=edep_t, edep_event=edep_ev, escaped_event=esc_ev,
                   counters=dict(zip(COUNTERS, (int(c) for c in counters))))
        if log_cap > 0:
            out.update(log=log, log_n=logn, log_fate=fate)
        if want_start:
            out["start"] = start
        if want_digest:
            out["digest"] = digest
        if want_margins:
            out["margin"] = margin[:, :log_cap] if log_cap else margin[:, :0]
            out["tail_margin"] = tail
        return out
