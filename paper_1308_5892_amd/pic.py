"""Thin ctypes binding of the C ABI in include/pic.h (libpic.so, gfx950 HIP).

The functions keep the ABI's names and only marshal arguments: every step of
the PIC cycle runs in the HIP kernels of libpic.so.  PyTorch supplies the
device arena and the stream.  There is no CPU fallback: if libpic.so is not
built, importing the library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

MAX_SPECIES = 4
PIC_OK, PIC_EINVAL, PIC_ECOURANT, PIC_ENOMEM, PIC_EDEVICE, PIC_EFLAG, PIC_ESTATE = 0, -1, -2, -3, -4, -5, -6
PIC_FP64_FORM, PIC_TRACK_IDS, PIC_FILTER_CURRENT, PIC_FARADAY4 = 1, 2, 4, 8
PIC_PROFILE_UNIFORM, PIC_PROFILE_HARRIS = 0, 1
PIC_FLAG_NONFINITE, PIC_FLAG_LOST = 1, 2
ERROR_NAMES = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_ECOURANT", -3: "PIC_ENOMEM",
               -4: "PIC_EDEVICE", -5: "PIC_EFLAG", -6: "PIC_ESTATE"}

EXPORTED = ["pic_plan", "pic_init", "pic_load_maxwell_juttner", "pic_set_harris_field", "pic_step",
            "pic_diag", "pic_get_particles", "pic_set_particles", "pic_get_fields", "pic_set_fields",
            "pic_sync", "pic_steps_done", "pic_free", "pic_last_error", "pic_set_timing",
            "pic_get_timing", "pic_autotune", "pic_field_spectrum", "pic_diag_noalloc"]


class pic_species(C.Structure):
    _fields_ = [("q_over_e", C.c_double), ("m_over_me", C.c_double)]


class pic_box(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("n_x", C.c_double), ("rho0", C.c_double),
                ("max_particles", C.c_int64 * MAX_SPECIES), ("tile", C.c_int32 * 3), ("walls", C.c_int32)]


class pic_config(C.Structure):
    _fields_ = [("n_boxes", C.c_int32), ("boxes", C.POINTER(pic_box)), ("n_species", C.c_int32),
                ("species", pic_species * MAX_SPECIES), ("dt", C.c_double),
                ("sort_interval", C.c_int32), ("flags", C.c_uint32), ("hist_bins", C.c_int32),
                ("hist_lo", C.c_double), ("hist_hi", C.c_double), ("headroom", C.c_double)]


class pic_mj(C.Structure):
    _fields_ = [("theta", C.c_double), ("gamma_beta", C.c_double), ("axis", C.c_int32)]


class pic_load_desc(C.Structure):
    _fields_ = [("box", C.c_int32), ("species_a", C.c_int32), ("species_b", C.c_int32),
                ("mj_a", pic_mj), ("mj_b", pic_mj), ("ppc", C.c_double), ("profile", C.c_int32),
                ("profile_axis", C.c_int32), ("centre", C.c_double), ("thickness", C.c_double),
                ("half_width", C.c_double), ("seed", C.c_uint64), ("stream", C.c_uint64)]


class pic_harris_field(C.Structure):
    _fields_ = [("box", C.c_int32), ("grad_axis", C.c_int32), ("field_axis", C.c_int32),
                ("n_sheets", C.c_int32), ("b0", C.c_double), ("thickness", C.c_double),
                ("centre", C.c_double * 2)]


class pic_diag_out(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64), ("W_E", C.c_double * 3), ("W_B", C.c_double * 3),
                ("K", C.c_double * MAX_SPECIES), ("P", (C.c_double * 3) * MAX_SPECIES),
                ("sum_gm1", C.c_double * MAX_SPECIES), ("n_particles", C.c_int64 * MAX_SPECIES),
                ("n_overflow", C.c_int64 * MAX_SPECIES), ("gauss_max", C.c_double),
                ("gauss_rms", C.c_double), ("flags", C.c_uint32)]


class pic_timing(C.Structure):
    _fields_ = [("push_launches", C.c_int64), ("push_ms", C.c_double), ("field_launches", C.c_int64),
                ("field_ms", C.c_double), ("sort_launches", C.c_int64), ("sort_ms", C.c_double)]


class pic_tune_result(C.Structure):
    _fields_ = [("ms_per_step", C.c_double), ("ms_per_step_default", C.c_double), ("trials", C.c_int32)]


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libpic.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1308_5892_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.pic_plan.argtypes = [C.POINTER(pic_config), C.POINTER(C.c_size_t)]
        L.pic_init.argtypes = [C.POINTER(pic_config), C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.pic_load_maxwell_juttner.argtypes = [C.c_void_p, C.POINTER(pic_load_desc)]
        L.pic_set_harris_field.argtypes = [C.c_void_p, C.POINTER(pic_harris_field)]
        L.pic_step.argtypes = [C.c_void_p, C.c_int]
        L.pic_diag.argtypes = [C.c_void_p, C.c_int, C.POINTER(pic_diag_out), C.c_void_p]
        L.pic_diag_noalloc.argtypes = [C.c_void_p, C.c_int, C.POINTER(pic_diag_out), C.c_void_p]
        L.pic_get_particles.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_int64)]
        L.pic_set_particles.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_int64]
        L.pic_get_fields.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
        L.pic_set_fields.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.pic_sync.argtypes = [C.c_void_p]
        L.pic_steps_done.argtypes = [C.c_void_p]
        L.pic_steps_done.restype = C.c_int64
        L.pic_free.argtypes = [C.c_void_p]
        L.pic_last_error.argtypes = [C.c_void_p]
        L.pic_last_error.restype = C.c_char_p
        L.pic_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.pic_get_timing.argtypes = [C.c_void_p, C.POINTER(pic_timing), C.c_int]
        L.pic_field_spectrum.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p]
        L.pic_autotune.argtypes = [C.POINTER(pic_config), C.POINTER(pic_load_desc), C.c_int, C.c_void_p, C.c_size_t,
                                   C.c_void_p, C.c_int, C.POINTER(pic_config), C.POINTER(pic_box),
                                   C.POINTER(pic_tune_result)]
        for name in EXPORTED:
            if name not in ("pic_steps_done", "pic_last_error"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != PIC_OK:
        msg = lib().pic_last_error(ctx).decode() if ctx else ""
        raise PicError(rc, msg)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------- ABI wrappers

def make_config(boxes, species, dt, sort_interval=0, fp64=False, track_ids=False, hist_bins=0,
                hist_lo=-4.0, hist_hi=3.0, headroom=0.0, filter_current=False, faraday4=False):
    """Build a pic_config.  boxes: dicts with n, n_x, rho0, max_particles[, tile];
    species: list of (q_over_e, m_over_me)."""
    arr = (pic_box * len(boxes))()
    for i, b in enumerate(boxes):
        arr[i].n[:] = list(b["n"])
        arr[i].n_x = b["n_x"]
        arr[i].rho0 = b["rho0"]
        mp = list(b["max_particles"]) + [0] * (MAX_SPECIES - len(b["max_particles"]))
        arr[i].max_particles[:] = [int(v) for v in mp]
        arr[i].tile[:] = list(b.get("tile", (4, 4, 4)))
        arr[i].walls = int(b.get("walls", 0))
    cfg = pic_config()
    cfg.n_boxes = len(boxes)
    cfg.boxes = C.cast(arr, C.POINTER(pic_box))
    cfg.n_species = len(species)
    for s, (q, m) in enumerate(species):
        cfg.species[s].q_over_e = q
        cfg.species[s].m_over_me = m
    cfg.dt = dt
    cfg.sort_interval = sort_interval
    cfg.flags = ((PIC_FP64_FORM if fp64 else 0) | (PIC_TRACK_IDS if track_ids else 0) |
                 (PIC_FILTER_CURRENT if filter_current else 0) | (PIC_FARADAY4 if faraday4 else 0))
    cfg.hist_bins = hist_bins
    cfg.hist_lo = hist_lo
    cfg.hist_hi = hist_hi
    cfg.headroom = headroom
    cfg._boxes_keepalive = arr
    return cfg


def pic_plan(cfg):
    n = C.c_size_t(0)
    _check(lib().pic_plan(C.byref(cfg), C.byref(n)))
    return n.value


def pic_init(cfg, arena_ptr, nbytes, stream_ptr):
    ctx = C.c_void_p()
    _check(lib().pic_init(C.byref(cfg), C.c_void_p(arena_ptr), nbytes, C.c_void_p(stream_ptr), C.byref(ctx)))
    return ctx


def pic_load_maxwell_juttner(ctx, desc):
    _check(lib().pic_load_maxwell_juttner(ctx, C.byref(desc)), ctx)


def pic_set_harris_field(ctx, h):
    _check(lib().pic_set_harris_field(ctx, C.byref(h)), ctx)


def pic_step(ctx, n):
    _check(lib().pic_step(ctx, int(n)), ctx)


def pic_diag(ctx, box, hist=None):
    out = pic_diag_out()
    rc = lib().pic_diag(ctx, int(box), C.byref(out), _ptr(hist))
    _check(rc, ctx)
    return out


def pic_diag_noalloc(ctx, box, hist=None):
    """pic_diag summed in the library's static device scratch (no allocation)."""
    out = pic_diag_out()
    rc = lib().pic_diag_noalloc(ctx, int(box), C.byref(out), _ptr(hist))
    _check(rc, ctx)
    return out


def pic_get_particles(ctx, box, species, capacity):
    x = np.zeros(3 * capacity)
    u = np.zeros(3 * capacity)
    ids = np.zeros(capacity, dtype=np.int32)
    n = C.c_int64(capacity)
    _check(lib().pic_get_particles(ctx, int(box), int(species), _ptr(x), _ptr(u), _ptr(ids), C.byref(n)), ctx)
    k = n.value
    return x[:3 * k].reshape(-1, 3), u[:3 * k].reshape(-1, 3), ids[:k]


def pic_set_particles(ctx, box, species, x, u, ids=None):
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    n = len(x) // 3
    idp = None if ids is None else np.ascontiguousarray(ids, dtype=np.int32)
    _check(lib().pic_set_particles(ctx, int(box), int(species), _ptr(x), _ptr(u), _ptr(idp), n), ctx)


def pic_get_fields(ctx, box, ncells):
    e = np.zeros(3 * ncells)
    b = np.zeros(3 * ncells)
    j = np.zeros(3 * ncells)
    _check(lib().pic_get_fields(ctx, int(box), _ptr(e), _ptr(b), _ptr(j)), ctx)
    return e, b, j


def pic_set_fields(ctx, box, e=None, b=None):
    e = None if e is None else np.ascontiguousarray(e, dtype=np.float64)
    b = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    _check(lib().pic_set_fields(ctx, int(box), _ptr(e), _ptr(b)), ctx)


def pic_sync(ctx):
    _check(lib().pic_sync(ctx), ctx)


def pic_steps_done(ctx):
    return lib().pic_steps_done(ctx)


def pic_set_timing(ctx, enable):
    """0 off, 1 (or True) every launch kind, 2 the push only."""
    _check(lib().pic_set_timing(ctx, int(enable)), ctx)


def pic_get_timing(ctx, reset=True):
    t = pic_timing()
    _check(lib().pic_get_timing(ctx, C.byref(t), int(bool(reset))), ctx)
    return {"push_launches": t.push_launches, "push_ms": t.push_ms, "field_launches": t.field_launches,
            "field_ms": t.field_ms, "sort_launches": t.sort_launches, "sort_ms": t.sort_ms}


def pic_field_spectrum(ctx, box, n, field, comp, normal_axis):
    """Plane-summed power spectrum as an (N2, N1) array: [m2, m1]."""
    a1, a2 = [a for a in range(3) if a != normal_axis]
    ps = np.zeros(n[a1] * n[a2])
    _check(lib().pic_field_spectrum(ctx, int(box), int(field), int(comp), int(normal_axis), _ptr(ps)), ctx)
    return ps.reshape(n[a2], n[a1])


def pic_autotune(cfg, loads, arena_ptr, nbytes, stream_ptr, steps):
    """Returns (tuned pic_config, its pic_box array, pic_tune_result)."""
    arr = (pic_load_desc * max(1, len(loads)))(*loads)
    boxes = (pic_box * cfg.n_boxes)()
    out = pic_config()
    res = pic_tune_result()
    _check(lib().pic_autotune(C.byref(cfg), C.cast(arr, C.POINTER(pic_load_desc)), len(loads), C.c_void_p(arena_ptr),
                              nbytes, C.c_void_p(stream_ptr), int(steps), C.byref(out),
                              C.cast(boxes, C.POINTER(pic_box)), C.byref(res)))
    out._boxes_keepalive = boxes
    return out, boxes, res


def pic_free(ctx):
    _check(lib().pic_free(ctx))


def load_desc(box, species_a, species_b, mj_a, mj_b, ppc, seed, stream=0, profile=PIC_PROFILE_UNIFORM,
              profile_axis=0, centre=0.0, thickness=1.0, half_width=1.0):
    """mj_a/mj_b: (theta, gamma_beta, axis)."""
    d = pic_load_desc()
    d.box, d.species_a, d.species_b = box, species_a, species_b
    d.mj_a.theta, d.mj_a.gamma_beta, d.mj_a.axis = mj_a
    d.mj_b.theta, d.mj_b.gamma_beta, d.mj_b.axis = mj_b
    d.ppc = ppc
    d.profile, d.profile_axis = profile, profile_axis
    d.centre, d.thickness, d.half_width = centre, thickness, half_width
    d.seed, d.stream = seed, stream
    return d


# --------------------------------------------------- torch-backed simulation

def autotune(boxes, species, dt, loads, steps=10, **kw):
    """pic_autotune with a torch arena on the current device and torch's current
    stream.  loads: pic_load_desc list.  Returns (boxes with the chosen tiles,
    sort interval, {"ms_per_step", "ms_per_step_default", "trials"})."""
    import torch
    cfg = make_config(boxes, species, dt, **kw)
    nbytes = pic_plan(cfg)
    arena = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (arena.data_ptr() + 255) & ~255
    out, arr, res = pic_autotune(cfg, loads, base, nbytes, torch.cuda.current_stream().cuda_stream, steps)
    del arena
    tuned = []
    for i, b in enumerate(boxes):
        t = dict(b)
        t["tile"] = tuple(arr[i].tile[:])
        t["walls"] = arr[i].walls
        tuned.append(t)
    return tuned, out.sort_interval, {"ms_per_step": res.ms_per_step, "ms_per_step_default": res.ms_per_step_default,
                                      "trials": res.trials}


class Simulation:
    """A pic context whose arena is a torch uint8 tensor on the current device and
    whose stream is torch's current stream."""

    def __init__(self, boxes, species, dt, **kw):
        import torch
        self.cfg = make_config(boxes, species, dt, **kw)
        self.boxes = boxes
        self.nsp = len(species)
        self.nbytes = pic_plan(self.cfg)
        self.arena = torch.empty(self.nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.arena.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = torch.cuda.current_stream()
        self.ctx = pic_init(self.cfg, aligned, self.nbytes, self.stream.cuda_stream)

    def ncells(self, box=0):
        n = self.boxes[box]["n"]
        return int(n[0] * n[1] * n[2])

    def load(self, *a, **kw):
        pic_load_maxwell_juttner(self.ctx, load_desc(*a, **kw))

    def harris_field(self, box, grad_axis, field_axis, b0, thickness, centres):
        h = pic_harris_field()
        h.box, h.grad_axis, h.field_axis = box, grad_axis, field_axis
        h.n_sheets = len(centres)
        h.b0, h.thickness = b0, thickness
        for i, c in enumerate(centres):
            h.centre[i] = c
        pic_set_harris_field(self.ctx, h)

    def step(self, n=1):
        pic_step(self.ctx, n)

    def diag(self, box=0, hist_bins=0):
        hist = np.zeros(max(1, self.nsp * hist_bins), dtype=np.int64) if hist_bins else None
        o = pic_diag(self.ctx, box, hist)
        d = {"t": o.t, "step": o.step, "W_E": np.array(o.W_E[:]), "W_B": np.array(o.W_B[:]),
             "K": np.array(o.K[:self.nsp]), "P": np.array([o.P[s][:] for s in range(self.nsp)]),
             "sum_gm1": np.array(o.sum_gm1[:self.nsp]), "count": np.array(o.n_particles[:self.nsp]),
             "n_overflow": np.array(o.n_overflow[:self.nsp]), "gauss_max": o.gauss_max,
             "gauss_rms": o.gauss_rms, "flags": o.flags}
        if hist_bins:
            d["hist"] = hist.reshape(self.nsp, hist_bins)
        return d

    def particles(self, box=0, species=0):
        cap = int(self.boxes[box]["max_particles"][species])
        return pic_get_particles(self.ctx, box, species, max(cap, 1))

    def set_particles(self, box, species, x, u, ids=None):
        pic_set_particles(self.ctx, box, species, x, u, ids)

    def fields(self, box=0):
        return pic_get_fields(self.ctx, box, self.ncells(box))

    def spectrum(self, box=0, field=1, comp=1, normal_axis=1):
        return pic_field_spectrum(self.ctx, box, self.boxes[box]["n"], field, comp, normal_axis)

    def set_fields(self, box=0, e=None, b=None):
        pic_set_fields(self.ctx, box, e, b)

    def sync(self):
        pic_sync(self.ctx)

    def close(self):
        if self.ctx:
            pic_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
