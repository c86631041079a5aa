"""ctypes binding of libsph.so (argument marshalling only).

Every entry point of include/sph.h is exposed under the same name.  Device
buffers are torch tensors (PyTorch is used for device memory and streams);
this module only turns them into raw pointers and forwards the call.  There is
no fallback: if the HIP library is missing or fails to load, importing this
module raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
# the in-tree build, and only that one
LIB_PATH = os.path.join(PKG, "libsph.so")

SPH_OK, SPH_ERR_ARG, SPH_ERR_WORKSPACE, SPH_ERR_HIP, SPH_ERR_SCRATCH = 0, 1, 2, 3, 4
NOALLOC_SCRATCH_BYTES = 64 << 20
STATUS_N_ACTIVE, STATUS_MAX_NEIBS, STATUS_OVERFLOW, STATUS_DROPPED, STATUS_NONFINITE = 0, 1, 2, 3, 4
STATUS_WORDS = 8
NEIB_INDEX_BITS = 26
MAX_CAPACITY = 1 << NEIB_INDEX_BITS

EXPORTS = [
    "sph_status_string", "sph_abi_version", "sph_neib_list_entries", "sph_build_workspace_bytes",
    "sph_brick_shapes", "sph_neib_brick_entries", "sph_build_neighbors", "sph_forces", "sph_forces_workspace_bytes", "sph_integrate",
    "sph_dt_workspace_bytes", "sph_step_dt", "sph_count_interactions", "sph_integrate_backward",
    "sph_forces_backward_workspace_bytes", "sph_forces_backward", "sph_unpermute",
    "sph_diagnostics_workspace_bytes", "sph_reduce_diagnostics", "sph_count_missed_pairs",
    "sph_forces_noalloc", "sph_dt_scenes_workspace_bytes", "sph_step_dt_scenes", "sph_integrate_scenes",
    "sph_stream_copy", "sph_forces_corrector", "sph_forces_corrector_scenes",
]
MAX_SCENES = 1 << 20


class SphGrid(C.Structure):
    _fields_ = [("origin", C.c_double * 3), ("cell_size", C.c_float * 3), ("ncell", C.c_int32 * 3),
                ("periodic", C.c_uint32), ("cell_base", C.c_int32), ("cell_alpha", C.c_void_p),
                ("brick", C.c_int32 * 3)]


class SphParams(C.Structure):
    _fields_ = [("h", C.c_float), ("r_search", C.c_float), ("rho0", C.c_float), ("gamma", C.c_float),
                ("c0", C.c_float), ("alpha", C.c_float), ("eps_visc", C.c_float), ("nu", C.c_float),
                ("g", C.c_float * 3), ("cfl", C.c_float), ("visc_model", C.c_int32), ("delta", C.c_float),
                ("kernel", C.c_int32), ("formulation", C.c_int32)]


# sph_params.kernel / visc_model / formulation values (include/sph.h)
KERNEL_WENDLAND, KERNEL_CUBIC_SPLINE, KERNEL_QUADRATIC, KERNEL_GAUSSIAN = 0, 1, 2, 3
VISC_ARTIFICIAL, VISC_MORRIS, VISC_MONAGHAN_K = 0, 1, 2
FORM_GOLDEN_RULE, FORM_LANDRINI_MORRIS = 0, 1


class SphParticles(C.Structure):
    _fields_ = [("n", C.c_int32), ("capacity", C.c_int32), ("cell", C.c_void_p), ("pos", C.c_void_p),
                ("vel", C.c_void_p), ("info", C.c_void_p)]


class SphError(RuntimeError):
    pass


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsph.so is not built (%s): run `python -m paper_2207_11328_amd.build`" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    i32 = C.c_int32
    st = C.c_int
    L.sph_status_string.argtypes = [st]
    L.sph_status_string.restype = C.c_char_p
    L.sph_abi_version.argtypes = []
    L.sph_abi_version.restype = i32
    L.sph_neib_list_entries.argtypes = [i32, i32]
    L.sph_neib_list_entries.restype = C.c_size_t
    L.sph_forces_workspace_bytes.argtypes = [i32, i32]
    L.sph_forces_workspace_bytes.restype = C.c_size_t
    L.sph_build_workspace_bytes.argtypes = [i32, i32]
    L.sph_build_workspace_bytes.restype = C.c_size_t
    L.sph_neib_brick_entries.argtypes = [i32, i32]
    L.sph_neib_brick_entries.restype = C.c_size_t
    L.sph_brick_shapes.argtypes = [P, i32]
    L.sph_brick_shapes.restype = i32
    L.sph_build_neighbors.argtypes = [P, P, P, P, P, i32, P, P, P, P, P, P, C.c_size_t, P]
    L.sph_build_neighbors.restype = st
    L.sph_forces.argtypes = [P, P, P, P, P, i32, P, P, P, P, P, C.c_size_t, P]
    L.sph_forces.restype = st
    L.sph_forces_corrector.argtypes = [P, P, P, P, P, i32, P, P, P, P, P, P, P, P, C.c_size_t, P]
    L.sph_forces_corrector.restype = st
    L.sph_forces_corrector_scenes.argtypes = [P, P, P, P, P, i32, P, P, P, P, P, i32, P, P, P, P, C.c_size_t, P]
    L.sph_forces_corrector_scenes.restype = st
    L.sph_integrate.argtypes = [P, i32, P, P, P, P, P, P, P]
    L.sph_integrate.restype = st
    L.sph_dt_workspace_bytes.argtypes = []
    L.sph_dt_workspace_bytes.restype = C.c_size_t
    L.sph_step_dt.argtypes = [P, P, P, P, P, C.c_size_t, P]
    L.sph_step_dt.restype = st
    L.sph_dt_scenes_workspace_bytes.argtypes = [i32]
    L.sph_dt_scenes_workspace_bytes.restype = C.c_size_t
    L.sph_step_dt_scenes.argtypes = [P, P, P, P, P, i32, P, P, C.c_size_t, P]
    L.sph_step_dt_scenes.restype = st
    L.sph_integrate_scenes.argtypes = [P, P, i32, P, P, i32, P, P, P, P, P, P]
    L.sph_integrate_scenes.restype = st
    L.sph_count_interactions.argtypes = [P, P, P, P, P, i32, P, P]
    L.sph_count_interactions.restype = st
    L.sph_count_missed_pairs.argtypes = [P, P, P, P, P, i32, i32, P, P]
    L.sph_count_missed_pairs.restype = st
    L.sph_forces_noalloc.argtypes = [P, P, P, P, P, i32, P, P, P, P, P]
    L.sph_forces_noalloc.restype = st
    L.sph_stream_copy.argtypes = [P, P, C.c_size_t, i32, P]
    L.sph_stream_copy.restype = st
    L.sph_integrate_backward.argtypes = [P, i32, P, P, P, P, P, P, P, P]
    L.sph_integrate_backward.restype = st
    L.sph_forces_backward_workspace_bytes.argtypes = [i32, i32]
    L.sph_forces_backward_workspace_bytes.restype = C.c_size_t
    L.sph_forces_backward.argtypes = [P, P, P, P, P, i32, P, P, P, P, P, P, P, i32, P, C.c_size_t, P]
    L.sph_forces_backward.restype = st
    L.sph_unpermute.argtypes = [i32, P, P, P, P]
    L.sph_unpermute.restype = st
    L.sph_diagnostics_workspace_bytes.argtypes = []
    L.sph_diagnostics_workspace_bytes.restype = C.c_size_t
    L.sph_reduce_diagnostics.argtypes = [P, P, P, P, P, C.c_size_t, P]
    L.sph_reduce_diagnostics.restype = st
    return L


lib = _load()


def check(code: int, what: str):
    if code != SPH_OK:
        raise SphError("%s: %s" % (what, lib.sph_status_string(code).decode()))


def ptr(t) -> int | None:
    if t is None:
        return None
    assert t.is_contiguous(), "device buffers must be contiguous"
    return t.data_ptr()


def stream_ptr(stream=None) -> int | None:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def grid_struct(grid, cell_alpha=None, brick=None) -> SphGrid:
    """cell_alpha: optional device float tensor [n_cells] (per-cell alpha);
    brick: (bx, by, bz) of the LDS kernels, None for the default."""
    g = SphGrid()
    g.cell_alpha = ptr(cell_alpha)
    for d in range(3):
        g.brick[d] = 0 if brick is None else int(brick[d])
    for d in range(3):
        g.origin[d] = float(grid.origin[d])
        g.cell_size[d] = float(grid.cell_size[d])
        g.ncell[d] = int(grid.ncell[d])
    g.periodic = int(grid.periodic)
    g.cell_base = int(grid.cell_base)
    return g


def params_struct(p, alpha=None) -> SphParams:
    q = SphParams()
    q.h, q.r_search, q.rho0, q.gamma = p.h, p.r_search, p.rho0, p.gamma
    q.c0 = p.c0
    q.alpha = p.alpha if alpha is None else alpha
    q.eps_visc, q.nu = p.eps_visc, p.nu
    for d in range(3):
        q.g[d] = float(p.g[d])
    q.cfl = p.cfl
    q.visc_model = int(p.visc_model)
    q.delta = float(getattr(p, "delta", 0.0))
    q.kernel = int(getattr(p, "kernel", KERNEL_WENDLAND))
    q.formulation = int(getattr(p, "formulation", FORM_GOLDEN_RULE))
    return q


def particles_struct(n: int, cell, pos, vel, info) -> SphParticles:
    cap = cell.shape[0]
    assert pos.shape == (cap, 4) and vel.shape == (cap, 4) and info.shape == (cap,)
    assert cell.dtype == torch.int32 and pos.dtype == torch.float32 and vel.dtype == torch.float32
    assert info.dtype == torch.int32, "info is stored as int32 bits of the uint32 word"
    return SphParticles(int(n), int(cap), ptr(cell), ptr(pos), ptr(vel), ptr(info))


def sph_build_workspace_bytes(capacity: int, n_cells: int) -> int:
    return int(lib.sph_build_workspace_bytes(int(capacity), int(n_cells)))


def sph_neib_list_entries(capacity: int, max_neibs: int) -> int:
    return int(lib.sph_neib_list_entries(int(capacity), int(max_neibs)))


def sph_forces_workspace_bytes(capacity: int, n_cells: int) -> int:
    return int(lib.sph_forces_workspace_bytes(int(capacity), int(n_cells)))


def sph_dt_workspace_bytes() -> int:
    return int(lib.sph_dt_workspace_bytes())


def sph_neib_brick_entries(capacity: int, max_neibs: int) -> int:
    return int(lib.sph_neib_brick_entries(int(capacity), int(max_neibs)))


def sph_brick_shapes():
    """Supported brick shapes [(bx, by, bz), ...]; the first is the default."""
    k = int(lib.sph_brick_shapes(None, 0))
    buf = (C.c_int32 * (3 * k))()
    lib.sph_brick_shapes(buf, k)
    return [tuple(int(buf[3 * i + d]) for d in range(3)) for i in range(k)]


def sph_build_neighbors(grid: SphGrid, params: SphParams, parts: SphParticles, neibs, neib_count,
                        max_neibs: int, cell_start, cell_end, d_status, workspace, stream=None, perm_out=None,
                        neibs_brick=None):
    check(lib.sph_build_neighbors(C.byref(grid), C.byref(params), C.byref(parts), ptr(neibs), ptr(neib_count),
                                  int(max_neibs), ptr(cell_start), ptr(cell_end), ptr(d_status), ptr(perm_out),
                                  ptr(neibs_brick), ptr(workspace), workspace.numel() * workspace.element_size(),
                                  stream_ptr(stream)), "sph_build_neighbors")


def sph_forces(grid: SphGrid, params: SphParams, parts: SphParticles, neibs, neib_count, max_neibs: int,
               forces, workspace, stream=None, cell_start=None, cell_end=None, neibs_brick=None):
    check(lib.sph_forces(C.byref(grid), C.byref(params), C.byref(parts), ptr(neibs), ptr(neib_count),
                         int(max_neibs), ptr(cell_start), ptr(cell_end), ptr(neibs_brick), ptr(forces),
                         ptr(workspace), workspace.numel() * workspace.element_size(), stream_ptr(stream)),
          "sph_forces")


def sph_forces_corrector(grid: SphGrid, params: SphParams, star: SphParticles, neibs, neib_count, max_neibs: int,
                         d_dt, state_n: SphParticles, workspace, d_time=None, forces=None, stream=None,
                         cell_start=None, cell_end=None, neibs_brick=None):
    check(lib.sph_forces_corrector(C.byref(grid), C.byref(params), C.byref(star), ptr(neibs), ptr(neib_count),
                                   int(max_neibs), ptr(cell_start), ptr(cell_end), ptr(neibs_brick), ptr(d_dt),
                                   C.byref(state_n), ptr(d_time), ptr(forces), ptr(workspace),
                                   workspace.numel() * workspace.element_size(), stream_ptr(stream)),
          "sph_forces_corrector")


def sph_forces_corrector_scenes(grid: SphGrid, params: SphParams, star: SphParticles, neibs, neib_count,
                                max_neibs: int, d_dt, cell_scene, n_scenes: int, state_n: SphParticles, workspace,
                                d_time=None, forces=None, stream=None, cell_start=None, cell_end=None,
                                neibs_brick=None):
    check(lib.sph_forces_corrector_scenes(C.byref(grid), C.byref(params), C.byref(star), ptr(neibs),
                                          ptr(neib_count), int(max_neibs), ptr(cell_start), ptr(cell_end),
                                          ptr(neibs_brick), ptr(d_dt), ptr(cell_scene), int(n_scenes),
                                          C.byref(state_n), ptr(d_time), ptr(forces), ptr(workspace),
                                          workspace.numel() * workspace.element_size(), stream_ptr(stream)),
          "sph_forces_corrector_scenes")


def sph_forces_noalloc(grid: SphGrid, params: SphParams, parts: SphParticles, neibs, neib_count, max_neibs: int,
                       forces, stream=None, cell_start=None, cell_end=None, neibs_brick=None):
    check(lib.sph_forces_noalloc(C.byref(grid), C.byref(params), C.byref(parts), ptr(neibs), ptr(neib_count),
                                 int(max_neibs), ptr(cell_start), ptr(cell_end), ptr(neibs_brick), ptr(forces),
                                 stream_ptr(stream)), "sph_forces_noalloc")


def sph_integrate(params: SphParams, stage: int, d_dt, state_n: SphParticles, vel_star, forces,
                  out: SphParticles, d_time=None, stream=None):
    check(lib.sph_integrate(C.byref(params), int(stage), ptr(d_dt), C.byref(state_n), ptr(vel_star),
                            ptr(forces), C.byref(out), ptr(d_time), stream_ptr(stream)), "sph_integrate")


def sph_step_dt(params: SphParams, parts: SphParticles, forces, d_dt, workspace, stream=None):
    check(lib.sph_step_dt(C.byref(params), C.byref(parts), ptr(forces), ptr(d_dt), ptr(workspace),
                          workspace.numel() * workspace.element_size(), stream_ptr(stream)), "sph_step_dt")


def sph_dt_scenes_workspace_bytes(n_scenes: int) -> int:
    return int(lib.sph_dt_scenes_workspace_bytes(int(n_scenes)))


def sph_step_dt_scenes(grid: SphGrid, params: SphParams, parts: SphParticles, forces, cell_scene, n_scenes: int,
                       d_dt, workspace, stream=None):
    check(lib.sph_step_dt_scenes(C.byref(grid), C.byref(params), C.byref(parts), ptr(forces), ptr(cell_scene),
                                 int(n_scenes), ptr(d_dt), ptr(workspace),
                                 workspace.numel() * workspace.element_size(), stream_ptr(stream)),
          "sph_step_dt_scenes")


def sph_integrate_scenes(grid: SphGrid, params: SphParams, stage: int, d_dt, cell_scene, n_scenes: int,
                         state_n: SphParticles, vel_star, forces, out: SphParticles, d_time=None, stream=None):
    check(lib.sph_integrate_scenes(C.byref(grid), C.byref(params), int(stage), ptr(d_dt), ptr(cell_scene),
                                   int(n_scenes), C.byref(state_n), ptr(vel_star), ptr(forces), C.byref(out),
                                   ptr(d_time), stream_ptr(stream)), "sph_integrate_scenes")


def sph_count_interactions(grid: SphGrid, params: SphParams, parts: SphParticles, neibs, neib_count,
                           max_neibs: int, d_count, stream=None):
    check(lib.sph_count_interactions(C.byref(grid), C.byref(params), C.byref(parts), ptr(neibs),
                                     ptr(neib_count), int(max_neibs), ptr(d_count), stream_ptr(stream)),
          "sph_count_interactions")


def sph_stream_copy(src, dst, nbytes: int, blocks_per_cu: int = 8, stream=None):
    check(lib.sph_stream_copy(ptr(src), ptr(dst), int(nbytes), int(blocks_per_cu), stream_ptr(stream)),
          "sph_stream_copy")


def sph_count_missed_pairs(grid: SphGrid, params: SphParams, parts: SphParticles, neibs, neib_count,
                           max_neibs: int, phase: int, d_missed, stream=None):
    check(lib.sph_count_missed_pairs(C.byref(grid), C.byref(params), C.byref(parts), ptr(neibs),
                                     ptr(neib_count), int(max_neibs), int(phase), ptr(d_missed),
                                     stream_ptr(stream)), "sph_count_missed_pairs")


def sph_forces_backward_workspace_bytes(capacity: int, n_cells: int) -> int:
    return int(lib.sph_forces_backward_workspace_bytes(int(capacity), int(n_cells)))


def sph_integrate_backward(params: SphParams, stage: int, d_dt, state_n: SphParticles, grad_pos, grad_vel,
                           grad_pos_star, grad_vel_star, grad_forces, stream=None):
    check(lib.sph_integrate_backward(C.byref(params), int(stage), ptr(d_dt), C.byref(state_n), ptr(grad_pos),
                                     ptr(grad_vel), ptr(grad_pos_star), ptr(grad_vel_star), ptr(grad_forces),
                                     stream_ptr(stream)), "sph_integrate_backward")


def sph_forces_backward(grid: SphGrid, params: SphParams, parts: SphParticles, neibs, neib_count, max_neibs: int,
                        grad_forces, grad_pos, grad_vel, grad_params, accumulate: bool, workspace, stream=None,
                        cell_start=None, cell_end=None, neibs_brick=None):
    check(lib.sph_forces_backward(C.byref(grid), C.byref(params), C.byref(parts), ptr(neibs), ptr(neib_count),
                                  int(max_neibs), ptr(cell_start), ptr(cell_end), ptr(neibs_brick),
                                  ptr(grad_forces), ptr(grad_pos), ptr(grad_vel), ptr(grad_params),
                                  1 if accumulate else 0, ptr(workspace),
                                  workspace.numel() * workspace.element_size(), stream_ptr(stream)),
          "sph_forces_backward")


def sph_unpermute(n: int, perm, src, dst, stream=None):
    check(lib.sph_unpermute(int(n), ptr(perm), ptr(src), ptr(dst), stream_ptr(stream)), "sph_unpermute")


def sph_diagnostics_workspace_bytes() -> int:
    return int(lib.sph_diagnostics_workspace_bytes())


def sph_reduce_diagnostics(params: SphParams, parts: SphParticles, forces, d_out, workspace, stream=None):
    check(lib.sph_reduce_diagnostics(C.byref(params), C.byref(parts), ptr(forces), ptr(d_out), ptr(workspace),
                                     workspace.numel() * workspace.element_size(), stream_ptr(stream)),
          "sph_reduce_diagnostics")
