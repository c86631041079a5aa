"""Host-side checks of the C ABI (no GPU needed, no compute launched): the
library loads, exports every function include/sph.h declares, and the
ctypes structures match the C layout of the header."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    from paper_2207_11328_amd import abi as A
    return A


def test_every_declared_symbol_is_exported(abi):
    names = _declared()
    assert len(names) >= 9
    for nm in names:
        assert hasattr(abi.lib, nm), nm
    assert sorted(abi.EXPORTS) == names


def test_struct_layout_matches_header(abi, tmp_path):
    src = tmp_path / "layout.c"
    src.write_text("""
#include <stdio.h>
#include <stddef.h>
#include "sph.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(sph_grid), offsetof(sph_grid, cell_size), offsetof(sph_grid, periodic), offsetof(sph_grid, cell_base), offsetof(sph_grid, cell_alpha));
  printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(sph_params), offsetof(sph_params, g), offsetof(sph_params, visc_model),
         offsetof(sph_params, delta), offsetof(sph_params, kernel), offsetof(sph_params, formulation));
  printf("%zu %zu %zu %zu\\n", sizeof(sph_particles), offsetof(sph_particles, cell), offsetof(sph_particles, vel), offsetof(sph_particles, info));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    g = [int(v) for v in out[0].split()]
    assert g == [C.sizeof(abi.SphGrid), abi.SphGrid.cell_size.offset, abi.SphGrid.periodic.offset,
                 abi.SphGrid.cell_base.offset, abi.SphGrid.cell_alpha.offset]
    p = [int(v) for v in out[1].split()]
    assert p == [C.sizeof(abi.SphParams), abi.SphParams.g.offset, abi.SphParams.visc_model.offset,
                 abi.SphParams.delta.offset, abi.SphParams.kernel.offset, abi.SphParams.formulation.offset]
    q = [int(v) for v in out[2].split()]
    assert q == [C.sizeof(abi.SphParticles), abi.SphParticles.cell.offset, abi.SphParticles.vel.offset,
                 abi.SphParticles.info.offset]


def test_host_only_entry_points(abi):
    assert abi.lib.sph_abi_version() == 3
    for code in range(4):
        assert abi.lib.sph_status_string(code)
    a = abi.sph_build_workspace_bytes(1000, 500)
    b = abi.sph_build_workspace_bytes(2000, 500)
    c = abi.sph_build_workspace_bytes(1000, 5000)
    assert 0 < a < b and a < c
    assert a % 256 == 0
    assert abi.sph_dt_workspace_bytes() > 0
    assert abi.sph_dt_scenes_workspace_bytes(0) == 0
    assert abi.sph_dt_scenes_workspace_bytes(abi.MAX_SCENES + 1) == 0
    assert 0 < abi.sph_dt_scenes_workspace_bytes(1) < abi.sph_dt_scenes_workspace_bytes(128)


def test_brick_shapes(abi):
    shapes = abi.sph_brick_shapes()
    assert len(shapes) >= 1 and len(set(shapes)) == len(shapes), shapes
    assert all(len(s) == 3 and all(1 <= v <= 8 for v in s) for s in shapes), shapes


def test_argument_errors_return_before_any_launch(abi):
    """Null or inconsistent arguments are rejected synchronously."""
    g = abi.SphGrid()
    p = abi.SphParams()
    parts = abi.SphParticles(10, 5, None, None, None, None)  # n > capacity
    assert abi.lib.sph_forces(C.byref(g), C.byref(p), C.byref(parts), None, None, 128, None, None, None, None,
                              None, 0, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_forces(None, None, None, None, None, 128, None, None, None, None, None, 0,
                              None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_build_neighbors(None, None, None, None, None, 128, None, None, None, None, None, None, 0,
                                       None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_forces_backward(None, None, None, None, None, 128, None, None, None, None, None, None, None,
                                       0, None, 0, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_integrate_backward(None, 0, None, None, None, None, None, None, None,
                                          None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_forces_corrector(None, None, None, None, None, 128, None, None, None, None, None, None,
                                        None, None, 0, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_forces_corrector_scenes(None, None, None, None, None, 128, None, None, None, None, None, 1,
                                               None, None, None, None, 0, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_unpermute(-1, None, None, None, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_unpermute(0, None, None, None, None) == abi.SPH_OK
    assert abi.lib.sph_integrate(None, 0, None, None, None, None, None, None, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_integrate(C.byref(p), 2, None, None, None, None, None, None, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_step_dt(None, None, None, None, None, 0, None) == abi.SPH_ERR_ARG
    # per-scene steps: no table, or a scene count outside [1, SPH_MAX_SCENES]
    assert abi.lib.sph_step_dt_scenes(None, None, None, None, None, 1, None, None, 0, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_integrate_scenes(None, None, 0, None, None, 1, None, None, None, None, None,
                                        None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_count_interactions(None, None, None, None, None, 128, None, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_count_missed_pairs(None, None, None, None, None, 128, 0, None, None) == abi.SPH_ERR_ARG
    # a phase other than 0 or 1, and a missing output, on otherwise valid arguments
    g2 = abi.SphGrid()
    for d in range(3):
        g2.cell_size[d] = 0.06
        g2.ncell[d] = 4
    p2 = abi.SphParams()
    p2.h, p2.r_search, p2.rho0, p2.gamma, p2.c0 = 0.026, 0.06, 1000.0, 7.0, 20.0
    empty = abi.SphParticles(0, 0, None, None, None, None)
    table = (C.c_int32 * 64)()
    dts = (C.c_double * 2)()
    ws = (C.c_uint8 * 4096)()
    for bad in (0, abi.MAX_SCENES + 1):
        assert abi.lib.sph_step_dt_scenes(C.byref(g2), C.byref(p2), C.byref(empty), None, table, bad, dts, ws,
                                          4096, None) == abi.SPH_ERR_ARG
        assert abi.lib.sph_integrate_scenes(C.byref(g2), C.byref(p2), 0, dts, table, bad, C.byref(empty), None,
                                            None, C.byref(empty), None, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_step_dt_scenes(C.byref(g2), C.byref(p2), C.byref(empty), None, table, 2, dts, ws, 8,
                                      None) == abi.SPH_ERR_WORKSPACE
    assert abi.lib.sph_integrate_scenes(C.byref(g2), C.byref(p2), 2, dts, table, 2, C.byref(empty), None, None,
                                        C.byref(empty), None, None) == abi.SPH_ERR_ARG
    out = (C.c_longlong * 4)()
    for phase in (-1, 2):
        assert abi.lib.sph_count_missed_pairs(C.byref(g2), C.byref(p2), C.byref(empty), None, None, 128, phase,
                                              out, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_count_missed_pairs(C.byref(g2), C.byref(p2), C.byref(empty), None, None, 128, 0, None,
                                          None) == abi.SPH_ERR_ARG
    # the stream-copy probe: sizes and addresses off 16 bytes, missing
    # buffers, workgroups per CU outside 1..64; an empty copy launches nothing
    buf = (C.c_uint8 * 64)()
    al = (C.addressof(buf) + 15) & ~15
    assert abi.lib.sph_stream_copy(al, al + 16, 8, 8, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_stream_copy(al + 1, al + 16, 16, 8, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_stream_copy(None, al, 16, 8, None) == abi.SPH_ERR_ARG
    for bad in (0, 65):
        assert abi.lib.sph_stream_copy(al, al + 16, 16, bad, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_stream_copy(None, None, 0, 8, None) == abi.SPH_OK


def test_unknown_model_switches_are_rejected(abi):
    """An unknown kernel, laminar form or formulation is an argument error of
    sph_forces and sph_forces_backward; every known combination passes the
    parameter checks (and stops at the missing workspace, before any launch)."""
    g = abi.SphGrid()
    for d in range(3):
        g.cell_size[d] = 0.06
        g.ncell[d] = 4
    g.brick[:] = abi.sph_brick_shapes()[0]
    parts = abi.SphParticles(0, 0, None, None, None, None)
    gp = (C.c_double * 3)()

    def both(p):
        a = abi.lib.sph_forces(C.byref(g), C.byref(p), C.byref(parts), None, None, 128, None, None, None, None,
                               None, 0, None)
        b = abi.lib.sph_forces_backward(C.byref(g), C.byref(p), C.byref(parts), None, None, 128, None, None, None,
                                        None, None, None, gp, 0, None, 0, None)
        return a, b

    def params(**kw):
        p = abi.SphParams()
        p.h, p.r_search, p.rho0, p.gamma, p.c0 = 0.026, 0.06, 1000.0, 7.0, 20.0
        for k, v in kw.items():
            setattr(p, k, v)
        return p

    for kernel in range(4):
        for visc in range(3):
            for form in range(2):
                for delta in (0.0, 0.1):
                    assert both(params(kernel=kernel, visc_model=visc, formulation=form, delta=delta)) == \
                        (abi.SPH_ERR_WORKSPACE, abi.SPH_ERR_WORKSPACE)
    for bad in (dict(kernel=4), dict(kernel=-1), dict(visc_model=3), dict(formulation=2), dict(delta=-0.1)):
        assert both(params(**bad)) == (abi.SPH_ERR_ARG, abi.SPH_ERR_ARG), bad


def test_misaligned_brick_lists_are_rejected(abi):
    """The brick-local lists are written and read in 16-byte groups: a
    neibs_brick pointer that is not 16-byte aligned is an argument error of
    the build, the derivatives and the adjoint, returned before any launch
    (the device pointers below are placeholders that are never dereferenced)."""
    g = abi.SphGrid()
    for d in range(3):
        g.cell_size[d] = 0.06
        g.ncell[d] = 4
    g.brick[:] = abi.sph_brick_shapes()[0]
    p = abi.SphParams()
    p.h, p.r_search, p.rho0, p.gamma, p.c0 = 0.026, 0.06, 1000.0, 7.0, 20.0
    dev = C.c_void_p(0x100000)
    parts = abi.SphParticles(1, 1, dev, dev, dev, dev)
    gp = C.c_void_p(0x100000)
    big = C.c_size_t(1 << 40)
    # the same build call with no brick lists gets as far as the workspace check
    assert abi.lib.sph_build_neighbors(C.byref(g), C.byref(p), C.byref(parts), dev, dev, 128, dev, dev, dev,
                                       None, None, dev, C.c_size_t(0), None) == abi.SPH_ERR_WORKSPACE
    # the fused corrector: no step, or state n sharing storage with state *
    other = abi.SphParticles(1, 1, C.c_void_p(0x200000), C.c_void_p(0x200000), C.c_void_p(0x300000),
                             C.c_void_p(0x300000))
    assert abi.lib.sph_forces_corrector(C.byref(g), C.byref(p), C.byref(parts), dev, dev, 128, None, None, None,
                                        None, C.byref(other), None, None, dev, big, None) == abi.SPH_ERR_ARG
    assert abi.lib.sph_forces_corrector(C.byref(g), C.byref(p), C.byref(parts), dev, dev, 128, None, None, None,
                                        dev, C.byref(parts), None, None, dev, big, None) == abi.SPH_ERR_ARG
    short = abi.SphParticles(0, 1, C.c_void_p(0x200000), C.c_void_p(0x200000), C.c_void_p(0x300000),
                             C.c_void_p(0x300000))
    assert abi.lib.sph_forces_corrector(C.byref(g), C.byref(p), C.byref(parts), dev, dev, 128, None, None, None,
                                        dev, C.byref(short), None, None, dev, big, None) == abi.SPH_ERR_ARG
    for nb in (0x100002, 0x100008):
        nbp = C.c_void_p(nb)
        assert abi.lib.sph_build_neighbors(C.byref(g), C.byref(p), C.byref(parts), dev, dev, 128, dev, dev, dev,
                                           None, nbp, dev, big, None) == abi.SPH_ERR_ARG
        assert abi.lib.sph_forces(C.byref(g), C.byref(p), C.byref(parts), dev, dev, 128, dev, dev, nbp, dev, dev,
                                  big, None) == abi.SPH_ERR_ARG
        assert abi.lib.sph_forces_backward(C.byref(g), C.byref(p), C.byref(parts), dev, dev, 128, dev, dev, nbp,
                                           dev, dev, dev, gp, 0, dev, big, None) == abi.SPH_ERR_ARG


def test_weak_compressibility_check():
    """c0 >= 10 U with U the free-fall speed of the water height: the dam
    break's c0 = 20 m/s is below 10 sqrt(2 g 0.3) = 24.3 m/s (expected density
    variation about 1.5%); c0 = 30 m/s passes."""
    from paper_2207_11328_amd.checks import weak_compressibility
    from workloads import scenes as S
    p = S.sph_params(0.0043)
    r = weak_compressibility(p, 0.3)
    assert abs(r["U"] - (2 * 9.81 * 0.3) ** 0.5) < 1e-12
    assert not r["ok"] and 0.014 < r["density_variation"] < 0.015
    import dataclasses
    assert weak_compressibility(dataclasses.replace(p, c0=30.0), 0.3)["ok"]
    assert weak_compressibility(p, 0.0, u_max=3.0)["U"] == 3.0


def test_build_refuses_kernels_with_scratch():
    """The build step parses the compiler's kernel resource remarks and fails
    on any kernel with scratch memory, vector register spills or a dynamic
    stack (scalar spills go to vector lanes and are allowed)."""
    from paper_2207_11328_amd import build as Bd

    def remarks(name, scratch, vspill, sspill, dyn):
        pre = "x.hip:10:1: remark: "
        tail = " [-Rpass-analysis=kernel-resource-usage]"
        return "\n".join([pre + "Function Name: " + name + tail, "   10 | {", "      | ^",
                          pre + "    VGPRs: 128" + tail, pre + "    ScratchSize [bytes/lane]: %d" % scratch + tail,
                          pre + "    Dynamic Stack: %s" % dyn + tail, pre + "    SGPRs Spill: %d" % sspill + tail,
                          pre + "    VGPRs Spill: %d" % vspill + tail])

    ok = remarks("k_ok", 0, 0, 37, "False")
    u = Bd.resource_usage(ok)
    assert u == {"k_ok": {"VGPRs": "128", "ScratchSize [bytes/lane]": "0", "Dynamic Stack": "False",
                          "SGPRs Spill": "37", "VGPRs Spill": "0"}}
    Bd.check_no_scratch("x.hip", u)
    for bad in (remarks("k_bad", 8, 2, 0, "False"), remarks("k_bad", 0, 1, 0, "False"),
                remarks("k_bad", 0, 0, 0, "True")):
        with pytest.raises(Bd.ScratchError, match="k_bad"):
            Bd.check_no_scratch("x.hip", Bd.resource_usage(ok + "\n" + bad))
