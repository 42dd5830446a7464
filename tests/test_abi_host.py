"""The C-ABI library on the CPU: it loads, exports every function that
include/sale.h declares, and rejects invalid input in its host-side
validation before touching a device (no compute calls here)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2209_01983_amd import sale

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "sale.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sale_\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    L = sale.lib()
    decl = declared_functions()
    assert len(decl) >= 8
    for name in decl:
        assert hasattr(L, name), name
    assert sorted(sale.EXPORTS) == sorted(n for n in decl if n in sale.EXPORTS)
    assert set(decl) == set(sale.EXPORTS) | set(sale.POOL_EXPORTS)


def test_struct_layout_matches_header(tmp_path):
    """Size and every field offset of the ctypes mirrors equal what a C
    compiler makes of include/sale.h."""
    structs = {"sale_config": sale.sale_config, "sale_problem": sale.sale_problem}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(ny=-1), dict(nx=812, ny=812, nz=812), dict(gamma=1.0), dict(cfl=0.0), dict(cfl=1.0), dict(c_quad=-1.0),
    dict(t_end=-1.0), dict(precision=7), dict(hi=(0.0, 1.0, 1.0)), dict(remap_order=3),
    dict(remap_order=-1), dict(mode=2), dict(c_hg=-0.1), dict(c_hg=float("nan")),
    dict(mode=1, precision=1), dict(mode=1, remap_order=2),
])
def test_invalid_config_rejected(bad):
    kw = dict(nx=4, ny=4, nz=4)
    kw.update({k: v for k, v in bad.items() if k in ("nx", "ny", "nz")})
    rest = {k: v for k, v in bad.items() if k not in ("nx", "ny", "nz")}
    cfg = sale.make_config(kw["nx"], kw["ny"], kw["nz"], **rest)
    n = C.c_size_t(0)
    assert sale.lib().sale_workspace_bytes(C.byref(cfg), C.byref(n)) == sale.SALE_EINVAL
    rc, ctx = sale.sale_init(cfg, sale.sedov_problem(), 256, 1 << 30, 0)
    assert rc == sale.SALE_EINVAL and ctx is None


def test_workspace_bytes_scales_with_mesh():
    a = sale.sale_workspace_bytes(sale.make_config(16, 16, 16))
    b = sale.sale_workspace_bytes(sale.make_config(32, 32, 32))
    assert 6 < b / a < 9
    assert a % 256 == 0


def test_invalid_problems_rejected_before_device_work():
    cfg = sale.make_config(3, 2, 2)
    shapes = [(2, 2, 3), (2, 2, 3), (3, 3, 4), (3, 3, 4), (3, 3, 4)]
    good = [np.ones(s) for s in shapes]
    for which, val in ((0, np.nan), (0, -1.0), (1, -0.5), (1, np.inf), (2, np.nan)):
        arrs = [a.copy() for a in good]
        arrs[which].flat[3] = val
        p, keep = sale.user_problem(*arrs)
        rc, ctx = sale.sale_init(cfg, p, 256, 1 << 30, 0)
        assert rc == sale.SALE_EINVAL and ctx is None
    bad_sod = sale.sod_problem(rhoL=-1.0)
    assert sale.sale_init(cfg, bad_sod, 256, 1 << 30, 0)[0] == sale.SALE_EINVAL
    bad_sedov = sale.sedov_problem(edep=float("nan"))
    assert sale.sale_init(cfg, bad_sedov, 256, 1 << 30, 0)[0] == sale.SALE_EINVAL
    for kw in (dict(rho0=0.0), dict(p0=-1e-9), dict(u0=float("nan")), dict(dims=0), dict(dims=4)):
        assert sale.sale_init(cfg, sale.noh_problem(**kw), 256, 1 << 30, 0)[0] == sale.SALE_EINVAL, kw
    bad_kind = sale.sedov_problem()
    bad_kind.kind = 4
    assert sale.sale_init(cfg, bad_kind, 256, 1 << 30, 0)[0] == sale.SALE_EINVAL
    # misaligned or missing workspace, too small workspace
    ok = sale.sedov_problem()
    assert sale.sale_init(cfg, ok, 0, 1 << 30, 0)[0] == sale.SALE_EINVAL
    assert sale.sale_init(cfg, ok, 255, 1 << 30, 0)[0] == sale.SALE_EINVAL
    assert sale.sale_init(cfg, ok, 256, 1024, 0)[0] == sale.SALE_ENOMEM


def test_strerror_covers_every_code():
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert sale.sale_strerror(code) != "unknown code"
    assert sale.sale_strerror(99) == "unknown code"


def test_pool_create_rejects_invalid_arguments_before_device_work():
    big = 1 << 30
    assert sale.sale_pool_create(7, 4, 256, big, 0)[0] == sale.SALE_EINVAL        # precision
    assert sale.sale_pool_create(sale.SALE_FP64, 0, 256, big, 0)[0] == sale.SALE_EINVAL  # no slots
    assert sale.sale_pool_create(sale.SALE_FP64, 4, 0, big, 0)[0] == sale.SALE_EINVAL    # no arena
    assert sale.sale_pool_create(sale.SALE_FP64, 4, 128, big, 0)[0] == sale.SALE_EINVAL  # misaligned
    assert sale.sale_pool_create(sale.SALE_FP64, 4, 256, 512, 0)[0] == sale.SALE_ENOMEM  # header only
    L = sale.lib()
    out = C.c_int32(0)
    assert L.sale_pool_admit(None, None, None, 1, C.byref(out)) == sale.SALE_EINVAL
    assert L.sale_pool_advance(None, 1) == sale.SALE_EINVAL
    assert L.sale_pool_poll(None, None, 0, C.byref(out)) == sale.SALE_EINVAL
    assert L.sale_pool_fields(None, 0, 1, None, 0, 1) == sale.SALE_EINVAL
    assert L.sale_pool_release(None, 0) == sale.SALE_EINVAL
    L.sale_pool_destroy(None)
