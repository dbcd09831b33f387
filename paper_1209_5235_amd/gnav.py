"""ctypes binding of libgnav.so (argument marshalling only).

Every function keeps the C name and signature of include/gnav.h; all work
runs in the HIP library.  Device buffers are plain device pointers, e.g.
``tensor.data_ptr()`` of a torch tensor on the ROCm device; streams are raw
``hipStream_t`` values such as ``torch.cuda.current_stream().cuda_stream``.

The ``Context`` class is a convenience layer that marshals torch tensors
into those calls.  Importing this module fails loudly when the compiled
library is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgnav.so")

GNAV_OK = 0
STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "EGEOM", -5: "ESTATE",
          -6: "EUNSUPPORTED"}
COUNTERS = ["steps", "pe", "compton", "pair", "crossings", "escaped", "cutoff", "pushes", "stuck",
            "truncated", "tracks", "shortcuts", "dist_in", "dist_out", "inside", "voxel_nodes",
            "invalid", "dist_in_f32", "scored"] + \
    [f"{w}_{f}" for w in ("dist_in", "dist_out", "safety", "inside")
     for f in ("box", "tubs", "cons", "orb", "trd", "sphere")] + ["frame_maps"]
# distance arithmetic of ComputeStep (GNAV_PREC_*)
PREC_FP64, PREC_FP32_SCREENED, PREC_FP32 = 0, 1, 2
LIM_MOTHER, LIM_PE, LIM_COMPTON, LIM_PAIR, LIM_MAX_STEP = -1, -2, -3, -4, -5
NORMAL_NONE, NORMAL_FACE, NORMAL_EDGE = 0, 1, 2
NCOUNTERS = len(COUNTERS)
NOALLOC_MAX_SLOTS = 196608  # GNAV_NOALLOC_MAX_SLOTS: grid * block limit of gnav_transport_batch_noalloc
LOG_DTYPE = np.dtype([("touchable", np.int32), ("code", np.int32), ("step", np.float64),
                      ("edep", np.float64), ("energy", np.float64)])
DIGEST_DTYPE = np.dtype([("hash", np.uint64), ("n", np.int32), ("fate", np.int32),
                         ("sum_step", np.float64), ("sum_edep", np.float64)])

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)
_u8p = C.POINTER(C.c_uint8)


class gnav_geometry_desc(C.Structure):
    _fields_ = [
        ("n_solids", C.c_int32), ("solid_type", _i32p), ("solid_par", _f64p),
        ("n_mats", C.c_int32), ("mat_density", _f64p), ("mat_el_off", _i32p),
        ("el_Z", _i32p), ("el_A", _f64p), ("el_wfrac", _f64p),
        ("n_lv", C.c_int32), ("lv_solid", _i32p), ("lv_mat", _i32p), ("lv_dau_off", _i32p),
        ("lv_dau_cnt", _i32p), ("lv_voxelize", _u8p),
        ("n_pv", C.c_int32), ("pv_lv", _i32p), ("pv_rot", _f64p), ("pv_trans", _f64p),
        ("world_lv", C.c_int32), ("voxel_lists", C.c_int32),
    ]


class gnav_batch(C.Structure):
    _fields_ = [
        ("n_primaries", C.c_int64), ("event_dev", C.c_void_p), ("prim_id_dev", C.c_void_p),
        ("pos_dev", C.c_void_p), ("dir_dev", C.c_void_p), ("energy_dev", C.c_void_p),
        ("event_geom_dev", C.c_void_p), ("geom_id", C.c_int32), ("seed", C.c_uint64),
        ("e_cut", C.c_double), ("max_steps_per_track", C.c_int64), ("precision", C.c_int32),
        ("block", C.c_int32), ("grid", C.c_int32), ("count_work", C.c_int32),
        ("order", C.c_int32), ("record_dev", C.c_void_p), ("record_capacity", C.c_int64),
        ("record_count_dev", C.c_void_p), ("log_dev", C.c_void_p),
        ("log_capacity", C.c_int64), ("log_n_dev", C.c_void_p), ("log_fate_dev", C.c_void_p),
        ("chunk", C.c_int32), ("sort_period", C.c_int32), ("tuned", C.c_int32),
        ("digest_dev", C.c_void_p), ("keep_order", C.c_int32),
    ]


class gnav_step_outputs(C.Structure):
    _fields_ = [("step_dev", C.c_void_p), ("limiter_dev", C.c_void_p),
                ("next_touchable_dev", C.c_void_p), ("safety_dev", C.c_void_p),
                ("normal_dev", C.c_void_p), ("normal_valid_dev", C.c_void_p)]


class gnav_tuning(C.Structure):
    _fields_ = [("block", C.c_int32), ("grid", C.c_int32), ("chunk", C.c_int32),
                ("sort_period", C.c_int32), ("ms", C.c_float)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_1209_5235_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "gnav_create": ([C.c_int32, C.POINTER(P)], C.c_int32),
        "gnav_destroy": ([P], None),
        "gnav_last_error": ([P], C.c_char_p),
        "gnav_upload_geometry": ([P, C.POINTER(gnav_geometry_desc), _i32p, _i32p, P], C.c_int32),
        "gnav_touchables": ([P, C.c_int32, P, P, P, P], C.c_int32),
        "gnav_touchable_offset": ([P, C.c_int32, _i32p, _i32p], C.c_int32),
        "gnav_locate": ([P, C.c_int32, C.c_int64, P, P, P, C.c_int32, P], C.c_int32),
        "gnav_compute_step": ([P, C.c_int32, C.c_int64, P, P, P, P, P, P, P, C.c_int32, C.c_int32, P],
                              C.c_int32),
        "gnav_compute_step_ex": ([P, C.c_int32, C.c_int64, P, P, P, P, C.c_int32, C.c_int32,
                                  C.POINTER(gnav_step_outputs), P], C.c_int32),
        "gnav_compute_safety": ([P, C.c_int32, C.c_int64, P, P, P, C.c_int32, P], C.c_int32),
        "gnav_free_path": ([P, C.c_int32, C.c_int64, P, P, P, C.c_double, C.c_double, P, P, P],
                           C.c_int32),
        "gnav_tally_create": ([P, C.c_int32, C.POINTER(P)], C.c_int32),
        "gnav_tally_reset": ([P, P, P], C.c_int32),
        "gnav_tally_free": ([P, P], C.c_int32),
        "gnav_transport_batch": ([P, C.POINTER(gnav_batch), P, P], C.c_int32),
        "gnav_transport_batch_noalloc": ([P, C.POINTER(gnav_batch), P, P], C.c_int32),
        "gnav_read_tallies": ([P, P, P, P, P, P, P], C.c_int32),
        "gnav_autotune": ([P, C.POINTER(gnav_batch), P, C.c_int32, P, C.POINTER(gnav_tuning)],
                          C.c_int32),
        "gnav_graph_create": ([P, C.POINTER(gnav_batch), P, P, C.POINTER(P)], C.c_int32),
        "gnav_graph_launch": ([P, P, P], C.c_int32),
        "gnav_graph_free": ([P, P], C.c_int32),
        "gnav_mlp_create": ([P, C.c_int32, C.c_int32, P, C.POINTER(P)], C.c_int32),
        "gnav_mlp_n_params": ([P], C.c_int64),
        "gnav_mlp_grad": ([P, P, C.c_int64, P, P, P, P, P, P], C.c_int32),
        "gnav_mlp_adam": ([P, P, C.c_float, P], C.c_int32),
        "gnav_mlp_forward": ([P, P, C.c_int64, P, P, P, P], C.c_int32),
        "gnav_mlp_score": ([P, P, C.c_int64, P, P, P, P, P], C.c_int32),
        "gnav_mlp_get_params": ([P, P, P], C.c_int32),
        "gnav_mlp_free": ([P, P], C.c_int32),
        "gnav_ordering_classes": ([P, C.c_int32, _i32p], C.c_int32),
        "gnav_set_mlp": ([P, C.c_int32, P], C.c_int32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


lib = _load()

# --- thin wrappers with the C names ---------------------------------------
gnav_create = lib.gnav_create
gnav_destroy = lib.gnav_destroy
gnav_last_error = lib.gnav_last_error
gnav_upload_geometry = lib.gnav_upload_geometry
gnav_touchables = lib.gnav_touchables
gnav_touchable_offset = lib.gnav_touchable_offset
gnav_locate = lib.gnav_locate
gnav_compute_step = lib.gnav_compute_step
gnav_compute_step_ex = lib.gnav_compute_step_ex
gnav_compute_safety = lib.gnav_compute_safety
gnav_free_path = lib.gnav_free_path
gnav_tally_create = lib.gnav_tally_create
gnav_tally_reset = lib.gnav_tally_reset
gnav_tally_free = lib.gnav_tally_free
gnav_transport_batch = lib.gnav_transport_batch
gnav_transport_batch_noalloc = lib.gnav_transport_batch_noalloc
gnav_read_tallies = lib.gnav_read_tallies
gnav_autotune = lib.gnav_autotune
gnav_graph_create = lib.gnav_graph_create
gnav_graph_launch = lib.gnav_graph_launch
gnav_graph_free = lib.gnav_graph_free
gnav_mlp_create = lib.gnav_mlp_create
gnav_mlp_n_params = lib.gnav_mlp_n_params
gnav_mlp_grad = lib.gnav_mlp_grad
gnav_mlp_adam = lib.gnav_mlp_adam
gnav_mlp_forward = lib.gnav_mlp_forward
gnav_mlp_score = lib.gnav_mlp_score
gnav_mlp_get_params = lib.gnav_mlp_get_params
gnav_mlp_free = lib.gnav_mlp_free
gnav_ordering_classes = lib.gnav_ordering_classes
gnav_set_mlp = lib.gnav_set_mlp
CROSSING_DTYPE = np.dtype([("cls", np.int32), ("x", np.float32, 3), ("v", np.float32, 3),
                           ("label", np.int32)])


class GnavError(RuntimeError):
    pass


# --- convenience layer over torch tensors -----------------------------------

def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Context:
    """One library context on a device; owns uploaded geometries and tallies."""

    def __init__(self, device=0):
        h = C.c_void_p()
        st = gnav_create(int(device), C.byref(h))
        if st != GNAV_OK:
            raise GnavError(f"gnav_create failed: {STATUS.get(st, st)}")
        self.h = h
        self.device = device
        self.geoms = []
        self._keep = []

    def close(self):
        if getattr(self, "h", None) and gnav_destroy is not None:
            gnav_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()

    def _check(self, st, what):
        if st != GNAV_OK:
            msg = gnav_last_error(self.h).decode(errors="replace")
            raise GnavError(f"{what}: {STATUS.get(st, st)}: {msg}")

    def upload_geometry(self, desc, voxel_lists=0, stream=None):
        """Upload a workloads.GeometryDesc; returns (geom_id, n_touchables).  voxel_lists 0:
        shape-aware node lists, 1: bounding-box lists (gnav_geometry_desc.voxel_lists)."""
        arrs = dict(
            solid_type=_np(desc.solid_type, np.int32), solid_par=_np(desc.solid_par, np.float64),
            mat_density=_np(desc.mat_density, np.float64), mat_el_off=_np(desc.mat_el_off, np.int32),
            el_Z=_np(desc.el_Z, np.int32), el_A=_np(desc.el_A, np.float64),
            el_wfrac=_np(desc.el_wfrac, np.float64), lv_solid=_np(desc.lv_solid, np.int32),
            lv_mat=_np(desc.lv_mat, np.int32), lv_dau_off=_np(desc.lv_dau_off, np.int32),
            lv_dau_cnt=_np(desc.lv_dau_cnt, np.int32), lv_voxelize=_np(desc.lv_voxelize, np.uint8),
            pv_lv=_np(desc.pv_lv, np.int32), pv_rot=_np(desc.pv_rot, np.float64),
            pv_trans=_np(desc.pv_trans, np.float64),
        )

        def p(name, ct):
            a = arrs[name]
            return a.ctypes.data_as(C.POINTER(ct)) if a.size else None

        d = gnav_geometry_desc(
            desc.n_solids, p("solid_type", C.c_int32), p("solid_par", C.c_double),
            desc.n_mats, p("mat_density", C.c_double), p("mat_el_off", C.c_int32),
            p("el_Z", C.c_int32), p("el_A", C.c_double), p("el_wfrac", C.c_double),
            desc.n_lv, p("lv_solid", C.c_int32), p("lv_mat", C.c_int32),
            p("lv_dau_off", C.c_int32), p("lv_dau_cnt", C.c_int32), p("lv_voxelize", C.c_uint8),
            desc.n_pv, p("pv_lv", C.c_int32), p("pv_rot", C.c_double), p("pv_trans", C.c_double),
            int(desc.world_lv), int(voxel_lists))
        gid = C.c_int32()
        nt = C.c_int32()
        self._check(gnav_upload_geometry(self.h, C.byref(d), C.byref(gid), C.byref(nt),
                                         _stream(stream)), "gnav_upload_geometry")
        self.geoms.append((desc, nt.value))
        return gid.value, nt.value

    def touchables(self, geom_id):
        n = self.geoms[geom_id][1]
        out = [np.zeros(n, np.int32) for _ in range(4)]
        self._check(gnav_touchables(self.h, geom_id, *[o.ctypes.data_as(C.c_void_p) for o in out]),
                    "gnav_touchables")
        return out

    def touchable_offset(self, geom_id):
        off, tot = C.c_int32(), C.c_int32()
        self._check(gnav_touchable_offset(self.h, geom_id, C.byref(off), C.byref(tot)),
                    "gnav_touchable_offset")
        return off.value, tot.value

    def locate(self, geom_id, pos, dirs=None, out=None, stream=None, precision=0):
        import torch
        n = pos.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=pos.device)
        self._check(gnav_locate(self.h, geom_id, n, _ptr(pos), _ptr(dirs), _ptr(out), int(precision),
                                _stream(stream)), "gnav_locate")
        return out

    def compute_step(self, geom_id, pos, dirs, touch=None, with_next=True, stream=None, precision=0,
                     with_safety=False, max_step=None, learned=0, with_normal=False):
        """gnav_compute_step, or gnav_compute_step_ex when the safety or the normal is wanted;
        returns (step, limiter, next) followed by the safety when with_safety and by
        (normal [n][3], normal_valid) when with_normal."""
        import torch
        n = pos.shape[0]
        step = torch.empty(n, dtype=torch.float64, device=pos.device)
        lim = torch.empty(n, dtype=torch.int32, device=pos.device)
        nxt = torch.empty(n, dtype=torch.int32, device=pos.device) if with_next else None
        saf = torch.empty(n, dtype=torch.float64, device=pos.device) if with_safety else None
        nrm = torch.empty((n, 3), dtype=torch.float64, device=pos.device) if with_normal else None
        nval = torch.empty(n, dtype=torch.int32, device=pos.device) if with_normal else None
        if not with_safety and not with_normal:
            self._check(gnav_compute_step(self.h, geom_id, n, _ptr(pos), _ptr(dirs), _ptr(touch),
                                          _ptr(max_step), _ptr(step), _ptr(lim), _ptr(nxt),
                                          int(precision), int(learned), _stream(stream)),
                        "gnav_compute_step")
        else:
            out = gnav_step_outputs(step.data_ptr(), lim.data_ptr(),
                                    nxt.data_ptr() if nxt is not None else None,
                                    saf.data_ptr() if saf is not None else None,
                                    nrm.data_ptr() if nrm is not None else None,
                                    nval.data_ptr() if nval is not None else None)
            self._check(gnav_compute_step_ex(self.h, geom_id, n, _ptr(pos), _ptr(dirs), _ptr(touch),
                                             _ptr(max_step), int(precision), int(learned),
                                             C.byref(out), _stream(stream)), "gnav_compute_step_ex")
        res = (step, lim, nxt)
        if with_safety:
            res = res + (saf,)
        if with_normal:
            res = res + (nrm, nval)
        return res

    def free_path(self, geom_id, pos, dirs, life, energy=1.0, mu_mass=0.0, stream=None):
        """gnav_free_path: first interaction distances T and boundaries crossed."""
        import torch
        n = pos.shape[0]
        t = torch.empty(n, dtype=torch.float64, device=pos.device)
        nb = torch.empty(n, dtype=torch.int32, device=pos.device)
        self._check(gnav_free_path(self.h, geom_id, n, _ptr(pos), _ptr(dirs), _ptr(life), float(energy),
                                   float(mu_mass), _ptr(t), _ptr(nb), _stream(stream)), "gnav_free_path")
        return t, nb

    def compute_safety(self, geom_id, pos, touch=None, stream=None, precision=0):
        import torch
        n = pos.shape[0]
        out = torch.empty(n, dtype=torch.float64, device=pos.device)
        self._check(gnav_compute_safety(self.h, geom_id, n, _ptr(pos), _ptr(touch), _ptr(out),
                                        int(precision), _stream(stream)), "gnav_compute_safety")
        return out

    def tally_create(self, n_events):
        t = C.c_void_p()
        self._check(gnav_tally_create(self.h, int(n_events), C.byref(t)), "gnav_tally_create")
        return Tally(self, t, n_events)

    def ordering_classes(self, geom_id):
        n = C.c_int32()
        self._check(gnav_ordering_classes(self.h, geom_id, C.byref(n)), "gnav_ordering_classes")
        return n.value

    def set_mlp(self, geom_id, net):
        self._check(gnav_set_mlp(self.h, geom_id, net.h if net is not None else None),
                    "gnav_set_mlp")

    def _batch(self, geom_id, prim, seed=0, e_cut=1e-3, max_steps=0, precision=0, block=0, grid=0,
               log=None, event_geom=None, count_work=False, order=0, record=None, chunk=0,
               sort_period=0, tuned=False, digest=None, keep_order=False):
        b = gnav_batch()
        b.n_primaries = prim["energy"].shape[0]
        b.event_dev = prim["event"].data_ptr()
        b.prim_id_dev = prim["prim_id"].data_ptr()
        b.pos_dev = prim["pos"].data_ptr()
        b.dir_dev = prim["dir"].data_ptr()
        b.energy_dev = prim["energy"].data_ptr()
        b.event_geom_dev = event_geom.data_ptr() if event_geom is not None else None
        b.geom_id = geom_id
        b.seed = seed
        b.e_cut = e_cut
        b.max_steps_per_track = max_steps
        b.precision = precision
        b.block = block
        b.grid = grid
        b.count_work = int(bool(count_work))
        b.order = order
        b.chunk = chunk
        b.sort_period = sort_period
        b.tuned = int(bool(tuned))
        b.keep_order = int(bool(keep_order))
        if record is not None:
            b.record_dev = record["rec"].data_ptr()
            b.record_capacity = record["cap"]
            b.record_count_dev = record["count"].data_ptr()
        if digest is not None:
            b.digest_dev = digest.data_ptr()
        if log is not None:
            b.log_dev = log["rec"].data_ptr()
            b.log_capacity = log["cap"]
            b.log_n_dev = log["n"].data_ptr()
            b.log_fate_dev = log["fate"].data_ptr()
        return b

    def transport_batch(self, geom_id, prim, tally, stream=None, **kw):
        """prim: dict of device tensors event, prim_id, pos, dir, energy."""
        b = self._batch(geom_id, prim, **kw)
        self._check(gnav_transport_batch(self.h, C.byref(b), tally.h, _stream(stream)),
                    "gnav_transport_batch")

    def transport_batch_noalloc(self, geom_id, prim, tally, stream=None, **kw):
        """gnav_transport_batch_noalloc: the same transport with the library's fixed
        per-device scratch (allocates nothing)."""
        b = self._batch(geom_id, prim, **kw)
        self._check(gnav_transport_batch_noalloc(self.h, C.byref(b), tally.h, _stream(stream)),
                    "gnav_transport_batch_noalloc")

    def autotune(self, geom_id, prim, tally, trials=3, stream=None, **kw):
        """gnav_autotune: fastest {grid, chunk, sort_period} for this batch (cached in the
        context for batches passed with tuned=True)."""
        b = self._batch(geom_id, prim, **kw)
        out = gnav_tuning()
        self._check(gnav_autotune(self.h, C.byref(b), tally.h, int(trials), _stream(stream),
                                  C.byref(out)), "gnav_autotune")
        return dict(block=out.block, grid=out.grid, chunk=out.chunk, sort_period=out.sort_period,
                    ms=out.ms)

    def graph_create(self, geom_id, prim, tally, stream=None, **kw):
        b = self._batch(geom_id, prim, **kw)
        g = C.c_void_p()
        self._check(gnav_graph_create(self.h, C.byref(b), tally.h, _stream(stream), C.byref(g)),
                    "gnav_graph_create")
        return g

    def graph_launch(self, g, stream=None):
        self._check(gnav_graph_launch(self.h, g, _stream(stream)), "gnav_graph_launch")

    def graph_free(self, g):
        self._check(gnav_graph_free(self.h, g), "gnav_graph_free")


class MLP:
    """Candidate-ordering network on the device (parameters float32, products bf16 MFMA)."""

    PARAMS = ["w1x", "w1m", "b1", "w2", "b2", "w3", "b3"]

    def __init__(self, ctx, n_class, params, max_batch=4096):
        self.ctx = ctx
        self.n_class = n_class
        flat = np.concatenate([np.ascontiguousarray(params[k], np.float32).reshape(-1)
                               for k in self.PARAMS])
        h = C.c_void_p()
        ctx._check(gnav_mlp_create(ctx.h, int(n_class), int(max_batch),
                                   flat.ctypes.data_as(C.c_void_p), C.byref(h)), "gnav_mlp_create")
        self.h = h
        self.n_params = int(gnav_mlp_n_params(h))
        self.shapes = {k: np.asarray(params[k]).shape for k in self.PARAMS}

    def grad(self, x, cls, label, stream=None):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self.ctx._check(gnav_mlp_grad(self.ctx.h, self.h, x.shape[0], _ptr(x), _ptr(cls), _ptr(label),
                                      _ptr(g), _ptr(loss), _stream(stream)), "gnav_mlp_grad")
        return g, loss

    def step(self, x, cls, label, lr=1e-3, stream=None, want_loss=False):
        loss = None
        if want_loss:
            import torch
            loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self.ctx._check(gnav_mlp_grad(self.ctx.h, self.h, x.shape[0], _ptr(x), _ptr(cls), _ptr(label),
                                      None, _ptr(loss), _stream(stream)), "gnav_mlp_grad")
        self.ctx._check(gnav_mlp_adam(self.ctx.h, self.h, float(lr), _stream(stream)), "gnav_mlp_adam")
        return loss

    def forward(self, x, cls, stream=None):
        import torch
        out = torch.empty((x.shape[0], 64), dtype=torch.float32, device=x.device)
        self.ctx._check(gnav_mlp_forward(self.ctx.h, self.h, x.shape[0], _ptr(x), _ptr(cls), _ptr(out),
                                         _stream(stream)), "gnav_mlp_forward")
        return out

    def score(self, x, cls, stream=None):
        """gnav_mlp_score: the network as the transport evaluates it; (logits [n][64],
        predicted position [n])."""
        import torch
        n = x.shape[0]
        logits = torch.empty((n, 64), dtype=torch.float32, device=x.device)
        pred = torch.empty(n, dtype=torch.int32, device=x.device)
        self.ctx._check(gnav_mlp_score(self.ctx.h, self.h, n, _ptr(x), _ptr(cls), _ptr(logits), _ptr(pred),
                                       _stream(stream)), "gnav_mlp_score")
        return logits, pred

    def params(self):
        flat = np.zeros(self.n_params, np.float32)
        self.ctx._check(gnav_mlp_get_params(self.ctx.h, self.h, flat.ctypes.data_as(C.c_void_p)),
                        "gnav_mlp_get_params")
        out, o = {}, 0
        for k in self.PARAMS:
            n = int(np.prod(self.shapes[k]))
            out[k] = flat[o:o + n].reshape(self.shapes[k])
            o += n
        return out

    def unflatten(self, flat):
        out, o = {}, 0
        for k in self.PARAMS:
            n = int(np.prod(self.shapes[k]))
            out[k] = np.asarray(flat[o:o + n]).reshape(self.shapes[k])
            o += n
        return out

    def free(self):
        if self.h:
            gnav_mlp_free(self.ctx.h, self.h)
            self.h = None


class Tally:
    def __init__(self, ctx, h, n_events):
        self.ctx = ctx
        self.h = h
        self.n_events = n_events

    def reset(self, stream=None):
        self.ctx._check(gnav_tally_reset(self.ctx.h, self.h, _stream(stream)), "gnav_tally_reset")

    def read(self, stream=None):
        _, tot = self.ctx.touchable_offset(0)
        et = np.zeros(tot)
        ee = np.zeros(self.n_events)
        es = np.zeros(self.n_events)
        cn = np.zeros(NCOUNTERS, np.uint64)
        self.ctx._check(gnav_read_tallies(self.ctx.h, self.h, et.ctypes.data_as(C.c_void_p),
                                          ee.ctypes.data_as(C.c_void_p),
                                          es.ctypes.data_as(C.c_void_p),
                                          cn.ctypes.data_as(C.c_void_p), _stream(stream)),
                        "gnav_read_tallies")
        return dict(edep_touchable=et, edep_event=ee, escaped_event=es,
                    counters=dict(zip(COUNTERS, (int(c) for c in cn))))

    def free(self):
        if self.h:
            gnav_tally_free(self.ctx.h, self.h)
            self.h = None


def primaries_to_device(prim, device="cuda"):
    """Copy a workloads.Primaries set into device tensors."""
    import torch
    return dict(
        event=torch.from_numpy(np.ascontiguousarray(prim.event, np.int32)).to(device),
        prim_id=torch.from_numpy(np.ascontiguousarray(prim.prim_id, np.int32)).to(device),
        pos=torch.from_numpy(np.ascontiguousarray(prim.pos, np.float64)).to(device),
        dir=torch.from_numpy(np.ascontiguousarray(prim.dir, np.float64)).to(device),
        energy=torch.from_numpy(np.ascontiguousarray(prim.energy, np.float64)).to(device),
    )


def make_log(n_primaries, cap, device="cuda"):
    import torch
    return dict(rec=torch.zeros((3 * n_primaries, cap, 4), dtype=torch.float64, device=device),
                cap=cap, n=torch.zeros(3 * n_primaries, dtype=torch.int32, device=device),
                fate=torch.zeros(3 * n_primaries, dtype=torch.int32, device=device))


def make_digests(n_primaries, device="cuda"):
    """Zeroed per-track digests (3 slots per primary, 32 bytes each)."""
    import torch
    return torch.zeros((3 * n_primaries, 4), dtype=torch.float64, device=device)


def digests_to_numpy(d):
    return d.cpu().numpy().view(DIGEST_DTYPE).reshape(d.shape[0])


def make_recorder(capacity, device="cuda"):
    """Device buffers for the crossing recorder (32-byte records)."""
    import torch
    return dict(rec=torch.zeros((capacity, 8), dtype=torch.int32, device=device), cap=capacity,
                count=torch.zeros(1, dtype=torch.int64, device=device))


def recorder_to_numpy(rec):
    n = min(int(rec["count"].cpu()[0]), rec["cap"])
    return rec["rec"][:n].cpu().numpy().view(CROSSING_DTYPE).reshape(n)


def log_to_numpy(log):
    rec = log["rec"].cpu().numpy().view(LOG_DTYPE).reshape(log["n"].shape[0], log["cap"])
    return rec, log["n"].cpu().numpy(), log["fate"].cpu().numpy()
