"""The C-ABI library builds, loads and exports every symbol include/cdi.h
declares; host-only entry points behave (no device calls here)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "cdi.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(cdi_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2110_13055_amd import _lib as L
    lib = L.load()
    declared = _declared_symbols()
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    # the binding's signature table covers exactly the header
    assert sorted(L.SIGNATURES) == declared


def test_plan_is_host_only_and_sizes_workspaces():
    import paper_2110_13055_amd as P
    g, p, _ = P.preset("channel2d_128x64")
    info = P.plan(g, p)
    assert info.n_vox == 128 * 64
    assert info.n_prims > 0
    assert 0.6 * info.n_vox < info.n_fluid_est <= 0.7 * info.n_vox
    assert info.vox_bytes >= 9 * info.n_vox
    g, p, _ = P.preset("spheres3d_512")
    info = P.plan(g, p)
    assert abs(info.n_prims - 291440) < 100


def test_plan_rejects_bad_input():
    import paper_2110_13055_amd as P
    from paper_2110_13055_amd import _lib as L
    g, p, _ = P.preset("channel2d_128x64")
    p.tau = 0.5
    with pytest.raises(L.CdiError) as e:
        P.plan(g, p)
    assert e.value.code == L.E_UNSTABLE
    g, p, _ = P.preset("channel2d_128x64")
    g.dim = 4
    with pytest.raises(L.CdiError) as e:
        P.plan(g, p)
    assert e.value.code == L.E_INVALID
    # RSA cannot reach a porosity this low with this gap: the generator jams
    g, p, _ = P.preset("channel2d_128x64")
    g.porosity = 0.2
    with pytest.raises(L.CdiError) as e:
        P.plan(g, p)
    assert e.value.code == L.E_GEOMETRY


def test_moment_storage_needs_tau_one_and_no_body_force():
    import paper_2110_13055_amd as P
    from paper_2110_13055_amd import _lib as L
    g, p, _ = P.preset("channel2d_128x64", precision=L.MOMENTS)
    info = P.plan(g, p)
    f32 = P.plan(g, P.preset("channel2d_128x64")[1])
    assert info.node_bytes_per_fluid < f32.node_bytes_per_fluid  # no population planes
    p.tau = 0.8
    with pytest.raises(L.CdiError) as e:
        P.plan(g, p)
    assert e.value.code == L.E_INVALID and "tau = 1" in str(e.value)
    g, p, _ = P.preset("channel2d_128x64", precision=L.MOMENTS, drive=L.BODY_FORCE,
                       body_force=(1e-6, 0.0, 0.0))
    with pytest.raises(L.CdiError) as e:
        P.plan(g, p)
    assert e.value.code == L.E_INVALID


def test_last_error_is_a_string():
    from paper_2110_13055_amd import _lib as L
    lib = L.load()
    assert isinstance(lib.cdi_last_error(), bytes)


def test_struct_layouts_match_the_binding():
    """Every public struct has the size the ctypes mirror gives it (the
    loader checks this too); an unknown name is rejected."""
    import ctypes as C
    from paper_2110_13055_amd import _lib as L
    lib = L.load()
    for name, cls in L.STRUCTS.items():
        n = C.c_uint64()
        assert lib.cdi_struct_size(name.encode(), C.byref(n)) == L.OK
        assert n.value == C.sizeof(cls), name
    n = C.c_uint64()
    assert lib.cdi_struct_size(b"cdi_nothing", C.byref(n)) == L.E_INVALID
    assert lib.cdi_struct_size(None, C.byref(n)) == L.E_INVALID


@pytest.mark.parametrize("preset", ["channel2d_128x64", "spheres3d_64"])
@pytest.mark.parametrize("precision", [0, 1, 2, 3])
@pytest.mark.parametrize("streaming", [0, 1])
def test_plan_node_bytes_match_the_workspace_it_sizes(preset, precision, streaming):
    # the plan's per-node estimate (serving admission sizes requests with it)
    # against the exact node workspace for the planned node count (host only)
    import paper_2110_13055_amd as P
    from paper_2110_13055_amd import _lib as L
    g, p, _ = P.preset(preset, precision=precision, streaming=streaming)
    if precision == L.MOMENTS and streaming:
        pytest.skip("moment storage has no population arrays to stream")
    info = P.plan(g, p)
    nb = C.c_uint64()
    gc, _keep = g.to_c()
    pc = p.to_c()
    L.check(L.load().cdi_node_bytes(C.byref(gc), C.byref(pc), C.c_int64(info.n_fluid_est), C.byref(nb)),
            "cdi_node_bytes")
    bpf = info.node_bytes_per_fluid
    est = bpf * info.n_fluid_est
    # within 3 %, up to one 256-node tile of rounding and the per-instance scratch
    assert 0.97 * nb.value - 256 * bpf - 16384 <= est <= 1.05 * nb.value + 65536, (est, nb.value)
