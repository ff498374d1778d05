"""ctypes binding of the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps liboracle.so, a plain single-threaded C
implementation of the DSMC particle loop that shares no code with the GPU
library.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB, build as _build

_lib = None

STAGE_MOVE, STAGE_INJECT, STAGE_SORT, STAGE_COLLIDE, STAGE_SAMPLE = 1, 2, 4, 8, 16


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB):
        _build()
    lib = C.CDLL(LIB)
    P = C.c_void_p
    d, i, u32, i64 = C.c_double, C.c_int, C.c_uint32, C.c_int64
    lib.oracle_create.restype = P
    lib.oracle_create.argtypes = [i, P, i, P, i, P, P, P, i, P, P, P, P, P,
                                  d, d, d, d, d, d, u32, u32, i, i, i, i]
    lib.oracle_last_error.restype = C.c_char_p
    lib.oracle_set_alpha.argtypes = [P, d]
    lib.oracle_viscosity.restype = d
    lib.oracle_viscosity.argtypes = [P, d]
    lib.oracle_destroy.argtypes = [P]
    lib.oracle_init_fill.argtypes = [P, d, d, P]
    lib.oracle_step.argtypes = [P, i]
    lib.oracle_step_stages.argtypes = [P, i]
    lib.oracle_num_particles.restype = i64
    lib.oracle_num_particles.argtypes = [P]
    lib.oracle_get_particles.argtypes = [P, P, P, P, P]
    lib.oracle_set_particles.argtypes = [P, i64, P, P, P, P, u32, u32, P]
    lib.oracle_set_rotation.argtypes = [P, C.c_int, d]
    lib.oracle_inelastic_probability.argtypes = [P]
    lib.oracle_inelastic_probability.restype = d
    lib.oracle_get_rotation.argtypes = [P, P]
    lib.oracle_get_rot_sums.argtypes = [P, C.c_int, P]
    lib.oracle_rot_fields.argtypes = [P, C.c_int, P]
    lib.oracle_get_smax.argtypes = [P, P]
    lib.oracle_surface_sampling.argtypes = [P, C.c_int]
    lib.oracle_get_surface.argtypes = [P, P]
    lib.oracle_get_surface.restype = i64
    lib.oracle_get_surface_rot.argtypes = [P, P]
    lib.oracle_get_surface_rot.restype = i64
    lib.oracle_set_smax.argtypes = [P, P]
    lib.oracle_step_index.restype = u32
    lib.oracle_step_index.argtypes = [P]
    lib.oracle_next_pid.restype = u32
    lib.oracle_next_pid.argtypes = [P]
    lib.oracle_get_pair_counts.argtypes = [P, P, P]
    lib.oracle_get_counters.argtypes = [P, P]
    lib.oracle_get_sums.argtypes = [P, i, P]
    lib.oracle_num_steady.restype = i64
    lib.oracle_num_steady.argtypes = [P]
    lib.oracle_set_local_acc.argtypes = [P, P]
    lib.oracle_set_sums.argtypes = [P, i, P]
    lib.oracle_get_ewma_counts.argtypes = [P, P]
    lib.oracle_fields.argtypes = [P, i, P]
    lib.oracle_fields_of_sums.argtypes = [P, P, P, i, d, P]
    lib.oracle_get_volumes.argtypes = [P, P]
    lib.oracle_get_neighbours.argtypes = [P, P]
    lib.oracle_get_tets.argtypes = [P, P]
    lib.oracle_num_faces.argtypes = [P]
    lib.oracle_trace_one.argtypes = [P, P, P, i, u32, u32, d]
    lib.oracle_philox.argtypes = [P, P, P]
    lib.oracle_set_reference.argtypes = [P, d, d, P]
    for name in ["oracle_dig_sampled", "oracle_get_mprev"]:
        getattr(lib, name).argtypes = [P, P]
    lib.oracle_dig_gradients.argtypes = [P, P, P]
    lib.oracle_set_heat_relaxation.argtypes = [P, P]
    lib.oracle_dig_nsf.argtypes = [P, P, P, P]
    lib.oracle_dig_kn_cell.argtypes = [P, P, d, P]
    lib.oracle_dig_gate.argtypes = [P, P, P, P, d, i, P]
    lib.oracle_dig_solve.argtypes = [P, P, P, P, P]
    lib.oracle_dig_residual.argtypes = [P, P, P, P]
    lib.oracle_dig_face_hot.argtypes = [P, P, P, i, P]
    lib.oracle_dig_residual_faces.argtypes = [P, P, P, P]
    lib.oracle_dig_feedback.argtypes = [P, P, P, P]
    lib.oracle_dig_couple.argtypes = [P, P, P]
    _lib = lib
    return lib


class DigParams(C.Structure):
    _fields_ = [("kn_max", C.c_double), ("passes", C.c_int), ("n_m", C.c_int), ("eps_m", C.c_double),
                ("cfl", C.c_double), ("L0", C.c_double), ("feedback", C.c_int), ("global_dt", C.c_int),
                ("warm_start", C.c_int), ("unconverged", C.c_int), ("solver", C.c_int), ("krylov", C.c_int)]


class DigReport(C.Structure):
    _fields_ = [("iters", C.c_int), ("residual", C.c_double), ("converged", C.c_int), ("failed", C.c_int),
                ("n_rejected", C.c_int), ("n_reconstructed", C.c_int), ("n_unreached", C.c_int),
                ("np_before", C.c_int64), ("np_after", C.c_int64), ("fed_back", C.c_int), ("krylov_steps", C.c_int)]


def dig_params(kn_max=1.0, passes=3, n_m=200, eps_m=1e-6, cfl=0.5, L0=1.0, feedback=1, global_dt=0, warm_start=0,
               unconverged=0, solver=0, krylov=0):
    return DigParams(kn_max, passes, n_m, eps_m, cfl, L0, feedback, global_dt, warm_start, unconverged, solver,
                     krylov)


def _report_dict(r):
    return {k: getattr(r, k) for k, _ in DigReport._fields_}


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def philox(ctr, key):
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.oracle_philox(_p(c), _p(k), _p(out))
    return out


class Oracle:
    """One oracle simulation built from a workloads.Workload."""

    def __init__(self, wl, fill=True):
        lib = _load()
        self.lib = lib
        m, sp, run = wl.mesh, wl.species, wl.run
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        xyz = arr(m.xyz, np.float64)
        tets = arr(m.tets, np.int32)
        bf = arr(m.bfaces, np.int32)
        bg = arr(m.bgroup, np.int32)
        bp = arr(m.bpartner, np.int32) if m.bpartner is not None else None
        bcs = wl.boundaries
        gk = arr([b.kind for b in bcs], np.int32)
        gT = arr([b.T for b in bcs], np.float64)
        gu = arr([b.u for b in bcs], np.float64)
        gn = arr([b.n for b in bcs], np.float64)
        gs = arr([b.shift for b in bcs], np.float64)
        self.nt = int(tets.shape[0])
        self.nb = int(bf.shape[0])
        self.h = lib.oracle_create(
            int(xyz.shape[0]), _p(xyz), self.nt, _p(tets), int(bf.shape[0]), _p(bf), _p(bg), _p(bp),
            len(bcs), _p(gk), _p(gT), _p(gu), _p(gn), _p(gs),
            sp.mass, sp.d_ref, sp.omega, sp.T_ref, run.F_N, run.dt,
            run.seed & 0xFFFFFFFF, run.case_id, run.vel_fp32, run.n_ss, run.n_a, run.ewma_on)
        if not self.h:
            raise ValueError("oracle_create: " + lib.oracle_last_error().decode())
        if lib.oracle_set_alpha(self.h, float(sp.alpha)) != 0:
            raise ValueError("oracle_set_alpha: " + lib.oracle_last_error().decode())
        self.dr = int(getattr(sp, "dof_rot", 0))
        if lib.oracle_set_rotation(self.h, self.dr, float(getattr(sp, "z_rot", 0.0))) != 0:
            raise ValueError("oracle_set_rotation: " + lib.oracle_last_error().decode())
        if self.dr and getattr(sp, "a_heat", None) is not None:
            a = np.ascontiguousarray(sp.a_heat, np.float64)
            if lib.oracle_set_heat_relaxation(self.h, _p(a)) != 0:
                raise ValueError("oracle_set_heat_relaxation: singular matrix")
        # widths of the coupling arrays: primitives, HoT, sampled state, gradients
        self.nv, self.nh = (6, 12) if self.dr else (5, 9)
        self.nsw, self.ngw = (18, 15) if self.dr else (14, 12)
        self.wl = wl
        if fill:
            u0 = np.asarray(run.u0, dtype=np.float64)
            lib.oracle_init_fill(self.h, run.n0, run.T0, _p(u0))

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.oracle_destroy(self.h)
            self.h = None

    # -- stepping ---------------------------------------------------------
    def step(self, n=1):
        self.lib.oracle_step(self.h, n)

    def viscosity(self, T):
        return self.lib.oracle_viscosity(self.h, float(T))

    def step_stages(self, mask):
        self.lib.oracle_step_stages(self.h, mask)

    # -- state -------------------------------------------------------------
    @property
    def np(self):
        return int(self.lib.oracle_num_particles(self.h))

    def particles(self):
        n = self.np
        x = np.zeros((n, 3)); v = np.zeros((n, 3))
        c = np.zeros(n, np.int32); p = np.zeros(n, np.uint32)
        self.lib.oracle_get_particles(self.h, _p(x), _p(v), _p(c), _p(p))
        out = dict(x=x, v=v, cell=c, pid=p)
        if self.dr:
            ir = np.zeros(n)
            self.lib.oracle_get_rotation(self.h, _p(ir))
            out["ir"] = ir
        return out

    def set_particles(self, x, v, cell, pid, step, next_pid, ir=None):
        x = np.ascontiguousarray(x, np.float64); v = np.ascontiguousarray(v, np.float64)
        cell = np.ascontiguousarray(cell, np.int32); pid = np.ascontiguousarray(pid, np.uint32)
        ir = None if ir is None else np.ascontiguousarray(ir, np.float64)
        r = self.lib.oracle_set_particles(self.h, len(cell), _p(x), _p(v), _p(cell), _p(pid),
                                          step, next_pid, _p(ir))
        if r != 0:
            raise ValueError(self.lib.oracle_last_error().decode())

    @property
    def inelastic_probability(self):
        return self.lib.oracle_inelastic_probability(self.h)

    def rot_sums(self, which=0):
        o = np.zeros((self.nt, 4))
        self.lib.oracle_get_rot_sums(self.h, which, _p(o))
        return o

    def rot_fields(self, which=0):
        o = np.zeros((self.nt, 4))
        self.lib.oracle_rot_fields(self.h, which, _p(o))
        return o

    def surface_sampling(self, on=True):
        self.lib.oracle_surface_sampling(self.h, 1 if on else 0)

    def surface(self):
        """Surface sums [n_bfaces][5] (sum of v_in - v_out, of
        (|v_in|^2 - |v_out|^2)/2, hits) and the number of sampled steps."""
        o = np.zeros((self.nb, 5))
        n = self.lib.oracle_get_surface(self.h, _p(o))
        return o, int(n)

    def surface_rot(self):
        """Rotational energy given to each boundary face [n_bfaces] (a
        rotating gas) and the number of sampled steps."""
        o = np.zeros(self.nb)
        n = self.lib.oracle_get_surface_rot(self.h, _p(o))
        return o, int(n)

    def smax(self):
        o = np.zeros(self.nt)
        self.lib.oracle_get_smax(self.h, _p(o))
        return o

    def set_smax(self, a):
        a = np.ascontiguousarray(a, np.float64)
        self.lib.oracle_set_smax(self.h, _p(a))

    @property
    def step_index(self):
        return int(self.lib.oracle_step_index(self.h))

    @property
    def next_pid(self):
        return int(self.lib.oracle_next_pid(self.h))

    def pair_counts(self):
        a = np.zeros(self.nt, np.int32); b = np.zeros(self.nt, np.int32)
        self.lib.oracle_get_pair_counts(self.h, _p(a), _p(b))
        return a, b

    def counters(self):
        o = np.zeros(5, np.int64)
        self.lib.oracle_get_counters(self.h, _p(o))
        return dict(zip(["hops", "wall_hits", "injected", "removed", "lost"], o.tolist()))

    def sums(self, which=0):
        o = np.zeros((self.nt, 13))
        self.lib.oracle_get_sums(self.h, which, _p(o))
        return o

    def ewma_counts(self):
        o = np.zeros(self.nt, np.int32)
        self.lib.oracle_get_ewma_counts(self.h, _p(o))
        return o

    def set_sums(self, which, sums):
        a = np.ascontiguousarray(sums, np.float64)
        assert a.shape == (self.nt, 13)
        self.lib.oracle_set_sums(self.h, which, _p(a))

    @property
    def n_steady(self):
        return int(self.lib.oracle_num_steady(self.h))

    def set_local_acc(self, flags):
        f = np.ascontiguousarray(flags, np.uint8)
        self.lib.oracle_set_local_acc(self.h, _p(f))

    def fields(self, which=0):
        o = np.zeros((self.nt, 15))
        self.lib.oracle_fields(self.h, which, _p(o))
        return o

    def fields_of_sums(self, sums, vol, ns):
        """Fields [n][15] of given sums [n][13] over volumes [n], ns samples."""
        sums = np.ascontiguousarray(sums, np.float64)
        vol = np.ascontiguousarray(vol, np.float64)
        o = np.zeros((len(vol), 15))
        self.lib.oracle_fields_of_sums(self.h, _p(sums), _p(vol), len(vol), float(ns), _p(o))
        return o

    def volumes(self):
        o = np.zeros(self.nt)
        self.lib.oracle_get_volumes(self.h, _p(o))
        return o

    def neighbours(self):
        o = np.zeros((self.nt, 4), np.int32)
        self.lib.oracle_get_neighbours(self.h, _p(o))
        return o

    def tets(self):
        o = np.zeros((self.nt, 4), np.int32)
        self.lib.oracle_get_tets(self.h, _p(o))
        return o

    @property
    def n_faces(self):
        return int(self.lib.oracle_num_faces(self.h))

    def trace_one(self, x, v, cell, pid, step, t):
        x = np.array(x, np.float64); v = np.array(v, np.float64)
        c = self.lib.oracle_trace_one(self.h, _p(x), _p(v), int(cell), pid, step, t)
        return c, x, v

    # -- DIG coupling ------------------------------------------------------
    def set_reference(self, n0, T0, u0=(0.0, 0.0, 0.0)):
        u = np.asarray(u0, np.float64)
        self.lib.oracle_set_reference(self.h, n0, T0, _p(u))

    def dig_sampled(self):
        o = np.zeros((self.nt, self.nsw))
        self.lib.oracle_dig_sampled(self.h, _p(o))
        return o

    def dig_gradients(self, prim):
        prim = np.ascontiguousarray(prim, np.float64)
        o = np.zeros((self.nt, self.ngw))
        self.lib.oracle_dig_gradients(self.h, _p(prim), _p(o))
        return o

    def dig_nsf(self, prim, grad):
        prim = np.ascontiguousarray(prim, np.float64); grad = np.ascontiguousarray(grad, np.float64)
        o = np.zeros((self.nt, self.nh))
        self.lib.oracle_dig_nsf(self.h, _p(prim), _p(grad), _p(o))
        return o

    def dig_kn_cell(self, prim, L0=1.0):
        prim = np.ascontiguousarray(prim, np.float64)
        o = np.zeros(self.nt)
        self.lib.oracle_dig_kn_cell(self.h, _p(prim), L0, _p(o))
        return o

    def dig_gate(self, prim, hot, kn, kn_max, passes):
        prim = np.array(prim, np.float64, order="C"); hot = np.array(hot, np.float64, order="C")
        kn = np.ascontiguousarray(kn, np.float64)
        st = np.zeros(self.nt, np.int32)
        self.lib.oracle_dig_gate(self.h, _p(prim), _p(hot), _p(kn), kn_max, passes, _p(st))
        return prim, hot, st

    def dig_solve(self, prim, hot, **kw):
        prim = np.array(prim, np.float64, order="C"); hot = np.ascontiguousarray(hot, np.float64)
        prm = dig_params(**kw)
        rep = DigReport()
        self.lib.oracle_dig_solve(self.h, _p(prim), _p(hot), C.byref(prm), C.byref(rep))
        return prim, _report_dict(rep)

    def dig_face_hot(self, prim, hot, consistent=1):
        prim = np.ascontiguousarray(prim, np.float64); hot = np.ascontiguousarray(hot, np.float64)
        o = np.zeros((self.nt, 4, self.nh))
        self.lib.oracle_dig_face_hot(self.h, _p(prim), _p(hot), consistent, _p(o))
        return o

    def dig_residual_faces(self, prim, hotf):
        prim = np.ascontiguousarray(prim, np.float64); hotf = np.ascontiguousarray(hotf, np.float64)
        o = np.zeros((self.nt, self.nv))
        self.lib.oracle_dig_residual_faces(self.h, _p(prim), _p(hotf), _p(o))
        return o

    def dig_residual(self, prim, hot):
        prim = np.ascontiguousarray(prim, np.float64); hot = np.ascontiguousarray(hot, np.float64)
        o = np.zeros((self.nt, self.nv))
        self.lib.oracle_dig_residual(self.h, _p(prim), _p(hot), _p(o))
        return o

    def dig_feedback(self, prim_old, prim_new, state):
        a = np.ascontiguousarray(prim_old, np.float64); b = np.ascontiguousarray(prim_new, np.float64)
        st = np.ascontiguousarray(state, np.int32)
        self.lib.oracle_dig_feedback(self.h, _p(a), _p(b), _p(st))

    def dig_couple(self, **kw):
        prm = dig_params(**kw)
        rep = DigReport()
        self.lib.oracle_dig_couple(self.h, C.byref(prm), C.byref(rep))
        return _report_dict(rep)

    def mprev(self):
        o = np.zeros((self.nt, self.nv))
        self.lib.oracle_get_mprev(self.h, _p(o))
        return o
