"""Host-side checks of the C-ABI library (no GPU needed, no compute calls)."""

import math
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    return re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(swe_\w+)\s*\(", src, re.M)


HEADERS = sorted(f for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h"))


def test_library_exports_every_declared_symbol():
    from paper_1307_4839_amd import capi
    lib = capi.lib()
    assert "swe.h" in HEADERS and "swe_flowdir.h" in HEADERS
    names = [n for h in HEADERS for n in declared(h)]
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1307_4839_amd import capi
    names = {n for h in HEADERS for n in declared(h)}
    assert names <= set(capi.EXPORTS), names - set(capi.EXPORTS)


def test_flow_dir_validation_without_gpu():
    # argument checks happen on the host before any HIP call; an empty grid
    # is a no-op that launches nothing
    from paper_1307_4839_amd import capi
    for fn in (capi.swe_flow_dir_f32, capi.swe_flow_dir_f64):
        fn(0, 0, 5, 0, 0, 0)
        fn(0, 7, 0, 0, 0, 0)
        for args in ((0, 4, 4, 0, 0, 0),            # null buffers with cells
                     (16, -1, 4, 16, 0, 0),         # negative size
                     (16, 4, 4, 16, -1, 0),         # negative rows
                     (16, 4, 4, 16, 70000, 0),      # rows too large
                     (16, (1 << 30) + 4, 1, 16, 0, 0),
                     (16, 1 << 20, 1 << 17, 16, 0, 0)):  # more than 2^36 cells
            with pytest.raises(capi.SweError) as e:
                fn(*args)
            assert e.value.code == capi.SWE_EINVAL
    # a DEM not aligned to its element size (the address is never read)
    for fn, addr in ((capi.swe_flow_dir_f32, 4098), (capi.swe_flow_dir_f64, 4100)):
        with pytest.raises(capi.SweError) as e:
            fn(addr, 4, 4, 16, 0, 0)
        assert e.value.code == capi.SWE_EINVAL
    assert capi.swe_flow_dir_rows(8192, 8192, 4) == 11
    assert capi.swe_flow_dir_rows(14786, 10086, 4) == 24
    assert capi.swe_flow_dir_rows(8192, 8192, 8) == 4
    assert capi.swe_flow_dir_rows(3, 3, 4) == 4
    assert capi.swe_flow_dir_rows(1 << 16, 1 << 16, 4) == 64
    with pytest.raises(capi.SweError):
        capi.swe_flow_dir_rows(8, 8, 2)


def test_parameter_validation_without_gpu():
    # swe_workspace_bytes touches no device: it must validate on the host
    from paper_1307_4839_amd import capi
    ok = capi.make_params(10, 10, 1.0, 1.0)
    n = capi.swe_workspace_bytes(ok)
    assert n >= 6 * 100 * 8
    for bad in (capi.make_params(1, 10, 1.0, 1.0),
                capi.make_params(10, 10, 0.0, 1.0),
                capi.make_params(10, 10, 1.0, 1.0, bc=(0, 0, 0, 7)),
                capi.make_params(10, 10, 1.0, 1.0, fric_law=5),
                capi.make_params(10, 10, 1.0, 1.0, infil_on=1, dtheta=0.0),
                capi.make_params(10, 10, 1.0, 1.0, dt_max=0.0),
                # rows longer than 2^28 cells (a cell's byte offset within
                # its row must stay below 2^31)
                capi.make_params(capi.SWE_MAX_NX + 1, 2, 1.0, 1.0)):
        with pytest.raises(capi.SweError) as e:
            capi.swe_workspace_bytes(bad)
        assert e.value.code == capi.SWE_EINVAL
    # the longest row allowed
    assert capi.swe_workspace_bytes(capi.make_params(capi.SWE_MAX_NX, 2, 1.0, 1.0)) >= 6 * (1 << 29) * 8


def test_strerror_texts():
    from paper_1307_4839_amd import capi
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert capi.lib().swe_strerror(code)
    assert capi.lib().swe_strerror(-99) == b"unknown error"


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors must have the C layout: compile the header with gcc
    # and print every offset
    import ctypes as C
    import subprocess
    from paper_1307_4839_amd import capi
    checks = []
    for sname, cls in (("swe_params", capi.swe_params), ("swe_buffers", capi.swe_buffers),
                       ("swe_diag", capi.swe_diag)):
        checks.append((sname, "sizeof", C.sizeof(cls)))
        for f, _ in cls._fields_:
            checks.append((sname, f, getattr(cls, f).offset))
    body = "\n".join(
        f'printf("%zu\\n", (size_t)sizeof({s}));' if f == "sizeof"
        else f'printf("%zu\\n", (size_t)offsetof({s}, {f}));' for s, f, _ in checks)
    src = tmp_path / "layout.c"
    src.write_text("#include <stdio.h>\n#include <stddef.h>\n#include \"swe.h\"\n"
                   "int main(void){" + body + "return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == [v for _, _, v in checks]


def test_adjoint_rejects_rain_and_soil_fields_without_gpu():
    # the reverse pass has uniform rain and no infiltration: a buffer set
    # with any optional rain or soil field is refused before any device work
    # (the pointers below are never dereferenced)
    from paper_1307_4839_amd import capi
    p = capi.make_params(16, 16, 1.0, 1.0, fric_law=capi.SWE_FRIC_MANNING, fric_coef=0.03)
    for field in ("rain_w", "ks", "psi", "dtheta"):
        b = capi.swe_buffers()
        b.h = b.qx = b.qy = b.z = b.fric = 4096
        setattr(b, field, 4096)
        with pytest.raises(capi.SweError) as e:
            capi.swe_adj_create(p, b, 10, 3, 4096, 1, 5, 4096, 4096, 1 << 30, 0)
        assert e.value.code == capi.SWE_EINVAL


def test_adjoint_workspace_with_spacing_beyond_the_run_without_gpu():
    # a checkpoint spacing of at least the step count is one segment: the
    # workspace is that of a spacing equal to the step count, and it grows
    # with the spacing below it (one state and two rates per step kept)
    from paper_1307_4839_amd import capi
    p = capi.make_params(40, 24, 1.0, 1.0, fric_law=capi.SWE_FRIC_MANNING, fric_coef=0.03)
    one = capi.swe_adj_workspace_bytes(p, 60, 60, 3, 5)
    for ckpt in (61, 1000, 1 << 30):
        assert capi.swe_adj_workspace_bytes(p, 60, ckpt, 3, 5) == one
    sizes = [capi.swe_adj_workspace_bytes(p, 60, c, 3, 5) for c in (8, 15, 30, 60)]
    assert sizes == sorted(sizes) and len(set(sizes)) == 4
    plane = -(-40 * 24 * 8 // 256) * 256
    assert capi.swe_adj_workspace_bytes(p, 60, 60, 3, 5) - \
        capi.swe_adj_workspace_bytes(p, 60, 59, 3, 5) == 3 * plane * (3 - 1)


def test_first_order_limits_without_gpu():
    # the adjoint runs the second-order scheme only and the members of an
    # ensemble share it; an order outside {0, 1, 2} is invalid (all checked
    # before any device work)
    from paper_1307_4839_amd import capi
    for order in (-1, 3):
        with pytest.raises(capi.SweError):
            capi.swe_workspace_bytes(capi.make_params(8, 8, 1.0, 1.0, order=order))
    p1 = capi.make_params(16, 16, 1.0, 1.0, fric_law=capi.SWE_FRIC_MANNING, fric_coef=0.03,
                          order=1)
    b = capi.swe_buffers()
    b.h = b.qx = b.qy = b.z = b.fric = 4096
    with pytest.raises(capi.SweError) as e:
        capi.swe_adj_create(p1, b, 10, 3, 4096, 1, 5, 4096, 4096, 1 << 30, 0)
    assert e.value.code == capi.SWE_EINVAL
    p2 = capi.make_params(16, 16, 1.0, 1.0, fric_law=capi.SWE_FRIC_MANNING, fric_coef=0.03)
    with pytest.raises(capi.SweError) as e:
        capi.swe_batch_create([p2, p1], [b, b], 4096, 1 << 30, 0)
    assert e.value.code == capi.SWE_EINVAL


@pytest.mark.parametrize("flux", [1, 2, 3])
def test_flux_variant_limits_without_gpu(flux):
    # flux outside {0, 1, 2, 3} and a reconstruction outside {0, 1, 2} are
    # invalid; the members of an ensemble share one flux
    from paper_1307_4839_amd import capi
    for bad in (-1, 4):
        with pytest.raises(capi.SweError):
            capi.swe_workspace_bytes(capi.make_params(8, 8, 1.0, 1.0, flux=bad))
        with pytest.raises(capi.SweError):
            capi.swe_workspace_bytes(capi.make_params(8, 8, 1.0, 1.0, recon=bad - 1))
    for recon in (1, 2):
        capi.swe_workspace_bytes(capi.make_params(8, 8, 1.0, 1.0, recon=recon))
    capi.swe_workspace_bytes(capi.make_params(8, 8, 1.0, 1.0, flux=flux))
    p1 = capi.make_params(16, 16, 1.0, 1.0, fric_law=capi.SWE_FRIC_MANNING, fric_coef=0.03,
                          flux=flux)
    b = capi.swe_buffers()
    b.h = b.qx = b.qy = b.z = b.fric = 4096
    p2 = capi.make_params(16, 16, 1.0, 1.0, fric_law=capi.SWE_FRIC_MANNING, fric_coef=0.03)
    with pytest.raises(capi.SweError) as e:
        capi.swe_batch_create([p1, p2], [b, b], 4096, 1 << 30, 0)
    assert e.value.code == capi.SWE_EINVAL


def test_imposed_boundary_limits_without_gpu():
    # imposed depth finite and > 0, imposed discharge finite and >= 0 on the
    # sides that use them; other sides ignore the values; the adjoint
    # rejects imposed sides (ensembles take them)
    from paper_1307_4839_amd import capi
    H, Q, HQ = capi.SWE_BC_IMPOSED_H, capi.SWE_BC_IMPOSED_Q, capi.SWE_BC_IMPOSED_HQ
    good = [dict(bc=(H, Q, HQ, 0), bc_h=(1.0, 0.0, 0.5, -3.0), bc_q=(-1.0, 2.0, 0.0, math.nan)),
            dict(bc=(0, 1, Q, H), bc_h=(math.nan, 0, 0, 2.0), bc_q=(0, 0, 0.0, -1.0))]
    for kw in good:
        capi.swe_workspace_bytes(capi.make_params(8, 8, 1.0, 1.0, **kw))
    bad = [dict(bc=(H, 0, 0, 0), bc_h=(0.0, 1, 1, 1)),
           dict(bc=(0, HQ, 0, 0), bc_h=(1, -1.0, 1, 1), bc_q=(0, 1.0, 0, 0)),
           dict(bc=(0, 0, H, 0), bc_h=(1, 1, math.inf, 1)),
           dict(bc=(0, 0, 0, Q), bc_q=(0, 0, 0, -0.5)),
           dict(bc=(0, 0, 0, HQ), bc_h=(0, 0, 0, 1.0), bc_q=(0, 0, 0, math.nan)),
           dict(bc=(5, 0, 0, 0)),
           dict(bc=(0, -1, 0, 0))]
    for kw in bad:
        with pytest.raises(capi.SweError) as e:
            capi.swe_workspace_bytes(capi.make_params(8, 8, 1.0, 1.0, **kw))
        assert e.value.code == capi.SWE_EINVAL
    p1 = capi.make_params(16, 16, 1.0, 1.0, fric_law=capi.SWE_FRIC_MANNING, fric_coef=0.03,
                          bc=(Q, H, 0, 0), bc_h=(0, 1.0, 0, 0), bc_q=(0.5, 0, 0, 0))
    b = capi.swe_buffers()
    b.h = b.qx = b.qy = b.z = b.fric = 4096
    with pytest.raises(capi.SweError) as e:
        capi.swe_adj_create(p1, b, 10, 3, 4096, 1, 5, 4096, 4096, 1 << 30, 0)
    assert e.value.code == capi.SWE_EINVAL


def test_gauge_arguments_without_gpu():
    # a null context or negative sizes are refused before any device work
    from paper_1307_4839_amd import capi
    with pytest.raises(capi.SweError) as e:
        capi.swe_set_gauges(0, 4096, 3, 1, 4096, 10)
    assert e.value.code == capi.SWE_EINVAL
    with pytest.raises(capi.SweError) as e:
        capi.swe_get_gauges(0)
    assert e.value.code == capi.SWE_EINVAL


def test_boundary_value_arguments_without_gpu():
    from paper_1307_4839_amd import capi
    with pytest.raises(capi.SweError) as e:
        capi.swe_set_boundary_values(0, 0, 1.0, 1.0)
    assert e.value.code == capi.SWE_EINVAL
    with pytest.raises(capi.SweError) as e:
        capi.swe_batch_set_boundary_values(0, 0, 0, 1.0, 1.0)
    assert e.value.code == capi.SWE_EINVAL
