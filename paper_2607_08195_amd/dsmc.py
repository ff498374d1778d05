"""Thin Python binding of libdsmc.so (include/dsmc.h).

Argument marshalling only: every stage of the DSMC step runs in the HIP
kernels of the library.  PyTorch provides the device memory (through the
library's allocator callback, backed by torch's caching allocator) and the
HIP stream.  If the library is not built this module raises at import.
"""
import ctypes as C
import os

import numpy as np

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdsmc.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_2607_08195_amd.build.build() "
                      "(or __graft_entry__.build()) first")
_lib = C.CDLL(LIB_PATH)

STAGE_MOVE, STAGE_INJECT, STAGE_SORT, STAGE_COLLIDE, STAGE_SAMPLE = 1, 2, 4, 8, 16
SAMPLE_STEADY, SAMPLE_EWMA, SAMPLE_INSTANT = 0, 1, 2
STATUS = {0: "OK", -1: "INVALID", -2: "MESH", -3: "OOM", -4: "DEVICE", -5: "CAPACITY", -6: "LOST",
}

P = C.c_void_p


class MeshDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xyz", P), ("n_tets", C.c_int32), ("tet_vtx", P),
                ("n_bfaces", C.c_int32), ("bface_vtx", P), ("bface_group", P), ("bface_partner", P)]


class SpeciesDesc(C.Structure):
    _fields_ = [("mass", C.c_double), ("d_ref", C.c_double), ("omega", C.c_double), ("T_ref", C.c_double),
                ("alpha", C.c_double), ("dof_rot", C.c_int32), ("z_rot", C.c_double),
                ("heat_relax", C.c_double * 4)]


class BoundaryDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("T", C.c_double), ("u", C.c_double * 3), ("n", C.c_double),
                ("shift", C.c_double * 3)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", P)]


class RunDesc(C.Structure):
    _fields_ = [("n0", C.c_double), ("T0", C.c_double), ("u0", C.c_double * 3), ("F_N", C.c_double),
                ("dt", C.c_double), ("seed", C.c_uint64), ("case_id", C.c_uint32), ("vel_fp64", C.c_int32),
                ("n_ss", C.c_int32), ("n_a", C.c_int32), ("ewma_on", C.c_int32), ("fill", C.c_int32),
                ("capacity", C.c_int64), ("hip_stream", P), ("allocator", C.POINTER(Allocator))]


class State(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("x", P), ("v", P), ("cell", P), ("pid", P), ("smax", P),
                ("step", C.c_uint32), ("next_pid", C.c_uint32), ("ir", P)]


class MixedMeshDesc(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("xyz", P), ("n_cells", C.c_int32), ("cell_nv", P), ("cell_vtx", P),
                ("n_bfaces", C.c_int32), ("bface_nv", P), ("bface_vtx", P), ("bface_group", P),
                ("bface_partner", P)]


class TetMeshOut(C.Structure):
    _fields_ = [("n_vertices", C.c_int32), ("n_tets", C.c_int32), ("n_bfaces", C.c_int32), ("xyz", P),
                ("tet_vtx", P), ("tet_cell", P), ("bface_vtx", P), ("bface_group", P), ("bface_partner", P),
                ("bface_parent", P)]


class Counters(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("hops", C.c_int64), ("wall_hits", C.c_int64),
                ("injected", C.c_int64), ("removed", C.c_int64), ("lost", C.c_int64), ("step", C.c_uint32)]


class Tuning(C.Structure):
    _fields_ = [("move", C.c_int32), ("collide", C.c_int32), ("sort", C.c_int32), ("move_ms", C.c_double),
                ("collide_ms", C.c_double), ("sort_ms", C.c_double)]


class DigParams(C.Structure):
    _fields_ = [("kn_max", C.c_double), ("passes", C.c_int32), ("n_m", C.c_int32), ("eps_m", C.c_double),
                ("cfl", C.c_double), ("L0", C.c_double), ("feedback", C.c_int32), ("global_dt", C.c_int32),
                ("warm_start", C.c_int32), ("accel", C.c_int32), ("unconverged", C.c_int32),
                ("solver", C.c_int32), ("krylov", C.c_int32)]


class DigReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("residual", C.c_double), ("converged", C.c_int32), ("failed", C.c_int32),
                ("n_rejected", C.c_int32), ("n_reconstructed", C.c_int32), ("n_unreached", C.c_int32),
                ("np_before", C.c_int64), ("np_after", C.c_int64), ("n_closure", C.c_int32),
                ("n_fallback", C.c_int32), ("fed_back", C.c_int32), ("krylov_steps", C.c_int32)]


class MlpTrainParams(C.Structure):
    _fields_ = [("steps", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64)]


class MlpTrainReport(C.Structure):
    _fields_ = [("steps", C.c_int32), ("loss_first", C.c_double), ("loss_last", C.c_double)]


MLP_PARAMS = 35977
MLP_IN, MLP_OUT = 13, 9


DIG_OUT = {"sampled": (0, 14), "half": (1, 5), "new": (2, 5), "hot": (3, 9), "kn": (4, 1), "state": (5, 1),
           "mprev": (6, 5)}


def dig_params(kn_max=1.0, passes=3, n_m=200, eps_m=1e-6, cfl=0.5, L0=1.0, feedback=1, global_dt=0, warm_start=0,
               accel=0, unconverged=0, solver=0, krylov=0):
    return DigParams(kn_max, passes, n_m, eps_m, cfl, L0, feedback, global_dt, warm_start, accel, unconverged,
                     solver, krylov)


def _report(r):
    return {k: getattr(r, k) for k, _ in DigReport._fields_}


ctx_t = P
_lib.dsmc_init.argtypes = [C.POINTER(ctx_t), C.POINTER(MeshDesc), C.POINTER(SpeciesDesc), C.c_int32,
                           C.POINTER(BoundaryDesc), C.POINTER(RunDesc)]
_lib.dsmc_step.argtypes = [ctx_t, C.c_int32]
_lib.dsmc_step_stages.argtypes = [ctx_t, C.c_int32]
_lib.dsmc_sample.argtypes = [ctx_t, C.c_int32, P, C.c_int32]
_lib.dsmc_get_sums.argtypes = [ctx_t, C.c_int32, P, C.POINTER(C.c_int64)]
_lib.dsmc_get_rot_sums.argtypes = [ctx_t, C.c_int32, P, C.POINTER(C.c_int64)]
_lib.dsmc_mesh_decompose.argtypes = [C.POINTER(MixedMeshDesc), C.POINTER(TetMeshOut)]
_lib.dsmc_mesh_error.restype = C.c_char_p
_lib.dsmc_mesh_error.argtypes = []
_lib.dsmc_sample_cells.argtypes = [ctx_t, C.c_int32, C.c_int32, P, P]
_lib.dsmc_rot_sample.argtypes = [ctx_t, C.c_int32, P]
_lib.dsmc_get_state.argtypes = [ctx_t, C.POINTER(State)]
_lib.dsmc_set_state.argtypes = [ctx_t, C.POINTER(State)]
_lib.dsmc_get_pair_counts.argtypes = [ctx_t, P, P]
_lib.dsmc_stats.argtypes = [ctx_t, C.POINTER(Counters)]
_lib.dsmc_sync.argtypes = [ctx_t]
_lib.dsmc_set_local_acc.argtypes = [ctx_t, P]
_lib.dsmc_profile.argtypes = [ctx_t, C.c_int32]
_lib.dsmc_profile_read.argtypes = [ctx_t, P, P, C.c_int32]
_lib.dsmc_profile_read.restype = C.c_int32
_lib.dsmc_profile_name.argtypes = [C.c_int32]
_lib.dsmc_profile_name.restype = C.c_char_p
_lib.dsmc_philox.argtypes = [P, P, P, C.c_int64]
_lib.dsmc_device_copy.argtypes = [ctx_t, P, P, C.c_size_t]
_lib.dsmc_device_line_reads.argtypes = [ctx_t, P, C.c_size_t, P, C.c_int, C.c_int, C.c_int]
_lib.dsmc_last_error.argtypes = [ctx_t]
_lib.dsmc_last_error.restype = C.c_char_p
_lib.dsmc_destroy.argtypes = [ctx_t]
_lib.dig_couple.argtypes = [ctx_t, C.POINTER(DigParams), C.POINTER(DigReport)]
_lib.dig_get.argtypes = [ctx_t, C.c_int32, P]
_lib.dig_residual.argtypes = [ctx_t, P, P, P]
_lib.dig_solve.argtypes = [ctx_t, P, P, C.POINTER(DigParams), C.POINTER(DigReport)]
_lib.dig_feedback.argtypes = [ctx_t, P, P, P, C.POINTER(C.c_int64)]
_lib.dsmc_set_sums.argtypes = [ctx_t, C.c_int32, P, P]
_lib.dsmc_set_rot_sums.argtypes = [ctx_t, C.c_int32, P]
_lib.dsmc_batch_init.argtypes = [C.POINTER(ctx_t), C.c_int32, C.POINTER(MeshDesc), C.POINTER(SpeciesDesc),
                                 P, C.POINTER(BoundaryDesc), C.POINTER(RunDesc)]
_lib.dsmc_batch_cases.argtypes = [ctx_t, C.POINTER(C.c_int32), P]
_lib.dsmc_graph_step.argtypes = [ctx_t, C.c_int32]
_lib.dsmc_get_tuning.argtypes = [ctx_t, C.POINTER(Tuning)]
_lib.dsmc_set_tuning.argtypes = [ctx_t, C.POINTER(Tuning)]
_lib.dsmc_autotune.argtypes = [ctx_t, C.c_int32, C.POINTER(Tuning)]
_lib.dsmc_mlp_create.argtypes = [C.POINTER(P), P, C.POINTER(Allocator)]
_lib.dsmc_mlp_set_weights.argtypes = [P, P]
_lib.dsmc_mlp_get_weights.argtypes = [P, P]
_lib.dsmc_mlp_init_weights.argtypes = [P, C.c_uint64]
_lib.dsmc_mlp_forward.argtypes = [P, P, C.c_int64, P, C.c_int32]
_lib.dsmc_mlp_backward.argtypes = [P, P, P, C.c_int64, P, C.POINTER(C.c_double)]
_lib.dsmc_mlp_backward_noalloc.argtypes = [P, P, P, C.c_int64, P, P]
_lib.dsmc_mlp_adam_step.argtypes = [P, P, C.c_float, C.c_float, C.c_float, C.c_float]
_lib.dsmc_mlp_train.argtypes = [P, P, P, C.c_int64, C.POINTER(MlpTrainParams), C.POINTER(MlpTrainReport)]
_lib.dsmc_mlp_last_error.argtypes = [P]
_lib.dsmc_mlp_last_error.restype = C.c_char_p
_lib.dsmc_mlp_destroy.argtypes = [P]
_lib.dig_set_closure.argtypes = [ctx_t, P, C.c_double]
_lib.dig_closure_data.argtypes = [ctx_t, P, P, P]
_lib.dig_batch_enable.argtypes = [ctx_t, P]
_lib.dsmc_surface_sampling.argtypes = [ctx_t, C.c_int32]
_lib.dsmc_instant_sampling.argtypes = [ctx_t, C.c_int32]
_lib.dsmc_get_surface.argtypes = [ctx_t, P, P, C.POINTER(C.c_int64)]
_lib.dsmc_get_surface_rot.argtypes = [ctx_t, P, P, C.POINTER(C.c_int64)]
for _f in ["dsmc_init", "dsmc_step", "dsmc_step_stages", "dsmc_sample", "dsmc_get_sums", "dsmc_get_rot_sums",
           "dsmc_rot_sample", "dsmc_mesh_decompose", "dsmc_sample_cells", "dsmc_get_state",
           "dsmc_set_state", "dsmc_get_pair_counts", "dsmc_stats", "dsmc_sync", "dsmc_set_local_acc",
           "dsmc_profile", "dsmc_philox", "dsmc_device_copy", "dsmc_device_line_reads", "dig_couple", "dig_get", "dig_residual",
           "dig_solve", "dig_feedback", "dsmc_set_sums", "dsmc_set_rot_sums", "dsmc_mlp_create", "dsmc_mlp_set_weights",
           "dsmc_mlp_get_weights", "dsmc_mlp_forward", "dsmc_mlp_backward", "dsmc_mlp_adam_step", "dsmc_mlp_train",
           "dsmc_mlp_init_weights", "dsmc_mlp_backward_noalloc", "dig_set_closure", "dig_closure_data", "dig_batch_enable", "dsmc_surface_sampling", "dsmc_get_surface",
           "dsmc_get_surface_rot", "dsmc_instant_sampling", "dsmc_batch_init", "dsmc_batch_cases", "dsmc_graph_step",
           "dsmc_get_tuning", "dsmc_set_tuning", "dsmc_autotune"]:
    getattr(_lib, _f).restype = C.c_int32

EXPORTED = ["dsmc_init", "dsmc_step", "dsmc_step_stages", "dsmc_sample", "dsmc_get_sums", "dsmc_get_rot_sums",
            "dsmc_rot_sample", "dsmc_mesh_decompose", "dsmc_mesh_error", "dsmc_sample_cells", "dsmc_get_state",
            "dsmc_set_state", "dsmc_get_pair_counts", "dsmc_stats", "dsmc_sync", "dsmc_set_local_acc",
            "dsmc_profile", "dsmc_profile_read", "dsmc_profile_name", "dsmc_philox", "dsmc_device_copy",
            "dsmc_device_line_reads",
            "dsmc_last_error", "dsmc_destroy", "dig_couple", "dig_get", "dig_residual", "dig_solve",
            "dig_feedback", "dsmc_set_sums", "dsmc_set_rot_sums", "dsmc_mlp_create", "dsmc_mlp_set_weights",
            "dsmc_mlp_get_weights",
            "dsmc_mlp_forward", "dsmc_mlp_backward", "dsmc_mlp_backward_noalloc", "dsmc_mlp_adam_step",
            "dsmc_mlp_train", "dsmc_mlp_last_error",
            "dsmc_mlp_destroy", "dig_set_closure", "dig_closure_data", "dig_batch_enable", "dsmc_surface_sampling",
            "dsmc_get_surface", "dsmc_get_surface_rot", "dsmc_instant_sampling"]


class DsmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _p(a):
    return None if a is None else a.ctypes.data_as(P)


def _check(status, ctx=None):
    if status != 0:
        raise DsmcError(status, _lib.dsmc_last_error(ctx).decode())


def decompose(xyz, cells, bfaces, bgroup, bpartner=None):
    """Tetrahedral mesh of a mixed-element mesh (dsmc_mesh_decompose):
    cells and bfaces are vertex-index lists (4/5/6/8 and 3/4 entries).
    Returns a dict of xyz, tets, tet_cell, bfaces, bgroup, bpartner,
    bparent."""
    xyz = np.ascontiguousarray(xyz, np.float64)
    cnv = np.array([len(c) for c in cells], np.int32)
    cv = np.ascontiguousarray(np.concatenate([np.asarray(c, np.int32) for c in cells]) if cells else
                              np.zeros(0, np.int32))
    bnv = np.array([len(f) for f in bfaces], np.int32)
    bv = np.ascontiguousarray(np.concatenate([np.asarray(f, np.int32) for f in bfaces]) if bfaces else
                              np.zeros(0, np.int32))
    bg = np.ascontiguousarray(bgroup, np.int32)
    bp = None if bpartner is None else np.ascontiguousarray(bpartner, np.int32)
    d = MixedMeshDesc(len(xyz), _p(xyz), len(cells), _p(cnv), _p(cv), len(bfaces), _p(bnv), _p(bv), _p(bg), _p(bp))
    o = TetMeshOut()
    st = _lib.dsmc_mesh_decompose(C.byref(d), C.byref(o))
    if st != 0:
        raise DsmcError(st, _lib.dsmc_mesh_error().decode())
    out = dict(xyz=np.zeros((o.n_vertices, 3)), tets=np.zeros((o.n_tets, 4), np.int32),
               tet_cell=np.zeros(o.n_tets, np.int32), bfaces=np.zeros((o.n_bfaces, 3), np.int32),
               bgroup=np.zeros(o.n_bfaces, np.int32), bpartner=np.zeros(o.n_bfaces, np.int32),
               bparent=np.zeros(o.n_bfaces, np.int32))
    o.xyz, o.tet_vtx, o.tet_cell = _p(out["xyz"]), _p(out["tets"]), _p(out["tet_cell"])
    o.bface_vtx, o.bface_group = _p(out["bfaces"]), _p(out["bgroup"])
    o.bface_partner, o.bface_parent = _p(out["bpartner"]), _p(out["bparent"])
    st = _lib.dsmc_mesh_decompose(C.byref(d), C.byref(o))
    if st != 0:
        raise DsmcError(st, _lib.dsmc_mesh_error().decode())
    return out


def philox(ctr, key):
    """Philox4x32-10 on the device for counters ctr[n,4] and key[2]."""
    c = np.ascontiguousarray(np.atleast_2d(ctr), dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros_like(c)
    _check(_lib.dsmc_philox(_p(c), _p(k), _p(out), c.shape[0]))
    return out


class _TorchAllocator:
    """Device memory from torch's caching allocator, handed to the library
    through its allocator callback."""

    def __init__(self, device, stream):
        self.device = device
        self.stream = stream

        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, self.stream)
            except Exception:
                return None

        def _free(ptr, user):
            torch.cuda.caching_allocator_delete(ptr)

        self._a = ALLOC_FN(_alloc)
        self._f = FREE_FN(_free)
        self.desc = Allocator(self._a, self._f, None)


class Simulation:
    """A DSMC run on one GPU, built from a workloads.Workload."""

    def __init__(self, wl, device=0, capacity=0, fill=True, stream=None, torch_memory=True):
        """wl: one workloads.Workload, or a list of them for a batch of
        independent cases in one context (species and batch-wide settings
        from the first)."""
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the DSMC library runs on the GPU only")
        self.device = device
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._keep = []
        cases = list(wl) if isinstance(wl, (list, tuple)) else [wl]

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        meshes = (MeshDesc * len(cases))()
        nbc = np.zeros(len(cases), np.int32)
        allb = []
        runs = (RunDesc * len(cases))()
        self._alloc = _TorchAllocator(device, self.stream) if torch_memory else None
        for k, w in enumerate(cases):
            m, run = w.mesh, w.run
            xyz = arr(m.xyz, np.float64)
            tets = arr(m.tets, np.int32)
            bf = arr(m.bfaces, np.int32)
            bg = arr(m.bgroup, np.int32)
            bp = arr(m.bpartner, np.int32) if m.bpartner is not None else None
            meshes[k] = MeshDesc(xyz.shape[0], _p(xyz), tets.shape[0], _p(tets), bf.shape[0], _p(bf), _p(bg), _p(bp))
            nbc[k] = len(w.boundaries)
            allb.extend(w.boundaries)
            runs[k] = RunDesc(run.n0, run.T0, (C.c_double * 3)(*run.u0), run.F_N, run.dt, run.seed, run.case_id,
                              0 if run.vel_fp32 else 1, run.n_ss, run.n_a, run.ewma_on, 1 if fill else 0, capacity,
                              P(self.stream.cuda_stream), C.pointer(self._alloc.desc) if self._alloc else None)
        bcs = (BoundaryDesc * max(1, len(allb)))()
        for i, b in enumerate(allb):
            bcs[i] = BoundaryDesc(b.kind, b.T, (C.c_double * 3)(*b.u), b.n, (C.c_double * 3)(*b.shift))
        sp = cases[0].species
        sd = SpeciesDesc(sp.mass, sp.d_ref, sp.omega, sp.T_ref, sp.alpha, int(getattr(sp, "dof_rot", 0)),
                         float(getattr(sp, "z_rot", 0.0)),
                         (C.c_double * 4)(*getattr(sp, "a_heat", (0.0, 0.0, 0.0, 0.0))))
        self.dof_rot = int(getattr(sp, "dof_rot", 0))
        # widths of the coupling arrays: primitives, HoT, sampled values
        self.nv, self.nh, self.nsw = (6, 12, 18) if self.dof_rot else (5, 9, 14)
        self.ctx = ctx_t()
        if len(cases) == 1 and not isinstance(wl, (list, tuple)):
            _check(_lib.dsmc_init(C.byref(self.ctx), C.byref(meshes[0]), C.byref(sd), int(nbc[0]), bcs,
                                  C.byref(runs[0])))
        else:
            _check(_lib.dsmc_batch_init(C.byref(self.ctx), len(cases), meshes, C.byref(sd), _p(nbc), bcs, runs))
        self.nt = int(sum(int(w.mesh.tets.shape[0]) for w in cases))
        self.nb = int(sum(int(w.mesh.bfaces.shape[0]) for w in cases))
        self.wl = wl
        self.cases = cases

    def close(self):
        if getattr(self, "ctx", None):
            _lib.dsmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _c(self, status):
        _check(status, self.ctx)

    # -- stepping --------------------------------------------------------
    def step(self, n=1):
        self._c(_lib.dsmc_step(self.ctx, n))

    def graph_step(self, n=2):
        """n steps through a captured HIP graph (needs a non-default stream)."""
        self._c(_lib.dsmc_graph_step(self.ctx, n))

    def case_cells(self):
        n = C.c_int32()
        self._c(_lib.dsmc_batch_cases(self.ctx, C.byref(n), None))
        b = np.zeros(n.value + 1, np.int32)
        self._c(_lib.dsmc_batch_cases(self.ctx, C.byref(n), _p(b)))
        return b

    def tuning(self):
        t = Tuning()
        self._c(_lib.dsmc_get_tuning(self.ctx, C.byref(t)))
        return dict(move=t.move, collide=t.collide, sort=t.sort)

    def set_tuning(self, move, collide, sort):
        t = Tuning(move, collide, sort, 0.0, 0.0, 0.0)
        self._c(_lib.dsmc_set_tuning(self.ctx, C.byref(t)))

    def autotune(self, trial_steps=3):
        t = Tuning()
        self._c(_lib.dsmc_autotune(self.ctx, trial_steps, C.byref(t)))
        return {k: getattr(t, k) for k, _ in Tuning._fields_}

    def step_stages(self, mask):
        self._c(_lib.dsmc_step_stages(self.ctx, mask))

    def sync(self):
        self._c(_lib.dsmc_sync(self.ctx))

    # -- outputs ---------------------------------------------------------
    def fields(self, which=SAMPLE_STEADY, on_device=False):
        if on_device:
            out = torch.empty((self.nt, 15), dtype=torch.float64, device=f"cuda:{self.device}")
            self._c(_lib.dsmc_sample(self.ctx, which, P(out.data_ptr()), 1))
            return out
        out = np.zeros((self.nt, 15))
        self._c(_lib.dsmc_sample(self.ctx, which, _p(out), 0))
        return out

    def sums(self, which=SAMPLE_STEADY):
        out = np.zeros((self.nt, 13))
        ns = C.c_int64()
        self._c(_lib.dsmc_get_sums(self.ctx, which, _p(out), C.byref(ns)))
        return out, int(ns.value)

    def rot_sums(self, which=SAMPLE_STEADY):
        """Rotational sums [n_tets][4] (sum I_r, sum v_i I_r) and the sample count."""
        out = np.zeros((self.nt, 4))
        ns = C.c_int64()
        self._c(_lib.dsmc_get_rot_sums(self.ctx, which, _p(out), C.byref(ns)))
        return out, int(ns.value)

    def rot_fields(self, which=SAMPLE_STEADY):
        """Rotational temperature and heat flux [n_tets][4] (T_r, q_r)."""
        out = np.zeros((self.nt, 4))
        self._c(_lib.dsmc_rot_sample(self.ctx, which, _p(out)))
        return out

    def sample_cells(self, tet_cell, n_cells, which=SAMPLE_STEADY):
        """Fields [n_cells][15] of the cells of a mixed mesh (dsmc_sample_cells)."""
        tc = np.ascontiguousarray(tet_cell, np.int32)
        out = np.zeros((n_cells, 15))
        self._c(_lib.dsmc_sample_cells(self.ctx, which, int(n_cells), _p(tc), _p(out)))
        return out

    def state(self, particles=True):
        st = State()
        smax = np.zeros(self.nt)
        st.smax = _p(smax)
        self._c(_lib.dsmc_get_state(self.ctx, C.byref(st)))
        n = int(st.n_particles)
        res = dict(n=n, step=int(st.step), next_pid=int(st.next_pid), smax=smax)
        if particles:
            x = np.zeros((n, 3)); v = np.zeros((n, 3))
            c = np.zeros(n, np.int32); p = np.zeros(n, np.uint32)
            ir = np.zeros(n) if self.dof_rot else None
            st.x, st.v, st.cell, st.pid, st.ir = _p(x), _p(v), _p(c), _p(p), _p(ir)
            self._c(_lib.dsmc_get_state(self.ctx, C.byref(st)))
            res.update(x=x, v=v, cell=c, pid=p)
            if ir is not None:
                res["ir"] = ir
        return res

    def set_state(self, x, v, cell, pid, step, next_pid, smax=None, ir=None):
        x = np.ascontiguousarray(x, np.float64); v = np.ascontiguousarray(v, np.float64)
        cell = np.ascontiguousarray(cell, np.int32); pid = np.ascontiguousarray(pid, np.uint32)
        sm = np.ascontiguousarray(smax, np.float64) if smax is not None else None
        irs = np.ascontiguousarray(ir, np.float64) if ir is not None else None
        st = State(len(cell), _p(x), _p(v), _p(cell), _p(pid), _p(sm), step, next_pid, _p(irs))
        self._c(_lib.dsmc_set_state(self.ctx, C.byref(st)))

    def instant_sampling(self, on=True):
        """Keep the moment sums of each sampled step (SAMPLE_INSTANT)."""
        self._c(_lib.dsmc_instant_sampling(self.ctx, 1 if on else 0))

    def surface_sampling(self, on=True):
        """Start (clearing the sums) or stop surface sampling (include/dsmc.h)."""
        self._c(_lib.dsmc_surface_sampling(self.ctx, 1 if on else 0))

    def surface(self):
        """Surface sums [n_bfaces][5], fields [n_bfaces][6] (number flux,
        pressure, shear stress (3), heat flux) and the sampled step count."""
        sums = np.zeros((self.nb, 5))
        fields = np.zeros((self.nb, 6))
        n = C.c_int64()
        self._c(_lib.dsmc_get_surface(self.ctx, _p(sums), _p(fields), C.byref(n)))
        return sums, fields, int(n.value)

    def surface_rot(self):
        """Rotational energy given to each boundary face [n_bfaces] (J),
        the rotational heat flux into it [n_bfaces] (W/m^2) and the sampled
        step count (dsmc_get_surface_rot; a rotating gas)."""
        sums = np.zeros(self.nb)
        qr = np.zeros(self.nb)
        n = C.c_int64()
        self._c(_lib.dsmc_get_surface_rot(self.ctx, _p(sums), _p(qr), C.byref(n)))
        return sums, qr, int(n.value)

    def pair_counts(self):
        a = np.zeros(self.nt, np.int32); b = np.zeros(self.nt, np.int32)
        self._c(_lib.dsmc_get_pair_counts(self.ctx, _p(a), _p(b)))
        return a, b

    def stats(self):
        c = Counters()
        self._c(_lib.dsmc_stats(self.ctx, C.byref(c)))
        return dict(n_particles=c.n_particles, hops=c.hops, wall_hits=c.wall_hits, injected=c.injected,
                    removed=c.removed, lost=c.lost, step=c.step)

    def set_local_acc(self, flags):
        f = np.ascontiguousarray(flags, np.uint8)
        self._c(_lib.dsmc_set_local_acc(self.ctx, _p(f)))

    # -- profiling -------------------------------------------------------
    def profile(self, enable=True):
        self._c(_lib.dsmc_profile(self.ctx, 1 if enable else 0))

    def profile_read(self):
        ms = np.zeros(16); cnt = np.zeros(16, np.int64)
        n = _lib.dsmc_profile_read(self.ctx, _p(ms), _p(cnt), 16)
        return {_lib.dsmc_profile_name(i).decode(): (float(ms[i]), int(cnt[i])) for i in range(n)}

    def device_copy(self, dst, src, nbytes):
        self._c(_lib.dsmc_device_copy(self.ctx, P(dst), P(src), nbytes))

    def device_line_reads(self, table, nbytes, sink, share, iters, blocks):
        """Scattered 16-byte reads of 128-byte lines (dsmc_device_line_reads)."""
        self._c(_lib.dsmc_device_line_reads(self.ctx, P(table), nbytes, P(sink), share, iters, blocks))

    def set_sums(self, which, sums, counts=None):
        a = np.ascontiguousarray(sums, np.float64)
        if a.shape != (self.nt, 13):
            raise ValueError("sums must be [n_tets, 13]")
        m = np.ascontiguousarray(counts, np.int32) if counts is not None else None
        self._c(_lib.dsmc_set_sums(self.ctx, which, _p(a), _p(m)))

    # -- DIG coupling (include/dig.h) ------------------------------------
    def set_rot_sums(self, which, sums):
        """Replace the rotational sums of an accumulator (dsmc_set_rot_sums)."""
        sums = np.ascontiguousarray(sums, np.float64)
        self._c(_lib.dsmc_set_rot_sums(self.ctx, which, _p(sums)))

    def dig_couple(self, **kw):
        prm = dig_params(**kw)
        rep = DigReport()
        self._c(_lib.dig_couple(self.ctx, C.byref(prm), C.byref(rep)))
        return _report(rep)

    def dig_get(self, which):
        code, k = DIG_OUT[which]
        k = {5: self.nv, 9: self.nh, 14: self.nsw}.get(k, k)
        if which == "state":
            out = np.zeros(self.nt, np.int32)
        else:
            out = np.zeros((self.nt, k)) if k > 1 else np.zeros(self.nt)
        self._c(_lib.dig_get(self.ctx, code, _p(out)))
        return out

    def dig_residual(self, prim, hot):
        prim = np.ascontiguousarray(prim, np.float64); hot = np.ascontiguousarray(hot, np.float64)
        out = np.zeros((self.nt, self.nv))
        self._c(_lib.dig_residual(self.ctx, _p(prim), _p(hot), _p(out)))
        return out

    def dig_solve(self, prim, hot, **kw):
        prim = np.array(prim, np.float64, order="C"); hot = np.ascontiguousarray(hot, np.float64)
        prm = dig_params(**kw)
        rep = DigReport()
        self._c(_lib.dig_solve(self.ctx, _p(prim), _p(hot), C.byref(prm), C.byref(rep)))
        return prim, _report(rep)

    def dig_feedback(self, prim_old, prim_new, state):
        a = np.ascontiguousarray(prim_old, np.float64); b = np.ascontiguousarray(prim_new, np.float64)
        st = np.ascontiguousarray(state, np.int32)
        n = C.c_int64()
        self._c(_lib.dig_feedback(self.ctx, _p(a), _p(b), _p(st), C.byref(n)))
        return int(n.value)

    def dig_enable(self, enabled):
        """Batch: couple only the cases whose flag is true (all by default)."""
        e = np.ascontiguousarray(np.asarray(enabled, np.int32))
        self._c(_lib.dig_batch_enable(self.ctx, _p(e)))

    def set_closure(self, mlp, gate_tol=0.05):
        """Attach a trained Mlp as the HoT closure of dig_couple (None detaches)."""
        self._closure = mlp
        self._c(_lib.dig_set_closure(self.ctx, mlp.h if mlp is not None else None, gate_tol))

    def closure_data(self):
        x = np.zeros((self.nt, MLP_IN), np.float32)
        t = np.zeros((self.nt, MLP_OUT), np.float32)
        v = np.zeros(self.nt, np.uint8)
        self._c(_lib.dig_closure_data(self.ctx, _p(x), _p(t), _p(v)))
        return x, t, v.astype(bool)


class Mlp:
    """The learned HoT closure (include/mlp.h) on one GPU."""

    def __init__(self, device=0, stream=None, torch_memory=True):
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the MLP kernels run on the GPU only")
        torch.cuda.set_device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._alloc = _TorchAllocator(device, self.stream) if torch_memory else None
        self.h = P()
        st = _lib.dsmc_mlp_create(C.byref(self.h), P(self.stream.cuda_stream),
                                  C.pointer(self._alloc.desc) if self._alloc else None)
        if st != 0:
            raise DsmcError(st, _lib.dsmc_mlp_last_error(None).decode())

    def _c(self, status):
        if status != 0:
            raise DsmcError(status, _lib.dsmc_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            _lib.dsmc_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, p):
        a = np.ascontiguousarray(p, np.float32)
        if a.size != MLP_PARAMS:
            raise ValueError("expected 35977 parameters")
        self._c(_lib.dsmc_mlp_set_weights(self.h, _p(a)))

    def init_weights(self, seed=0):
        self._c(_lib.dsmc_mlp_init_weights(self.h, seed))

    def get_weights(self):
        a = np.zeros(MLP_PARAMS, np.float32)
        self._c(_lib.dsmc_mlp_get_weights(self.h, _p(a)))
        return a

    def forward(self, x):
        x = np.ascontiguousarray(x, np.float32)
        y = np.zeros((x.shape[0], MLP_OUT), np.float32)
        self._c(_lib.dsmc_mlp_forward(self.h, _p(x), x.shape[0], _p(y), 0))
        return y

    def backward(self, x, t):
        x = np.ascontiguousarray(x, np.float32); t = np.ascontiguousarray(t, np.float32)
        g = np.zeros(MLP_PARAMS, np.float32)
        loss = C.c_double()
        self._c(_lib.dsmc_mlp_backward(self.h, _p(x), _p(t), x.shape[0], _p(g), C.byref(loss)))
        return float(loss.value), g

    def backward_noalloc(self, x, t, grad, loss):
        """dsmc_mlp_backward_noalloc on device tensors (x [n,13], t [n,9],
        grad [35977] float32, loss [1] float64): enqueued on the network's
        stream, no allocation and no synchronisation."""
        for a, dt in ((x, torch.float32), (t, torch.float32), (grad, torch.float32), (loss, torch.float64)):
            if not (a.is_cuda and a.is_contiguous() and a.dtype == dt):
                raise ValueError("device tensors, contiguous, float32 (float64 for loss) expected")
        self._c(_lib.dsmc_mlp_backward_noalloc(self.h, P(x.data_ptr()), P(t.data_ptr()), x.shape[0],
                                               P(grad.data_ptr()), P(loss.data_ptr())))

    def adam_step(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        g = np.ascontiguousarray(grad, np.float32)
        self._c(_lib.dsmc_mlp_adam_step(self.h, _p(g), lr, beta1, beta2, eps))

    def train(self, x, t, steps, batch=0, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0):
        x = np.ascontiguousarray(x, np.float32); t = np.ascontiguousarray(t, np.float32)
        prm = MlpTrainParams(steps, batch, lr, beta1, beta2, eps, seed)
        rep = MlpTrainReport()
        self._c(_lib.dsmc_mlp_train(self.h, _p(x), _p(t), x.shape[0], C.byref(prm), C.byref(rep)))
        return dict(steps=rep.steps, loss_first=rep.loss_first, loss_last=rep.loss_last)
