"""The largest mesh the library accepts (811^3 cells: every field array stays
below 4 GiB, the bound of the step kernels' 32-bit in-plane offsets), through
the C ABI.

A Sod tube along x on 811^3 decouples exactly into identical x rows (the
y and z faces sweep no volume and the transverse forces cancel), so after a
few steps every one of the 811^2 rows, including the ones at the top of the
index range where the byte offsets come closest to 2^32, must equal every
other (bitwise away from the walls, to 1e-14 near them) and the FP64
oracle's 811 x 4 x 4 tube to 1e-12 (MIXED32: 5e-6); mass and energy are
conserved.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2209_01983_amd import sale

from parity import TOL64, say  # noqa: E402

pytestmark = pytest.mark.gpu

N = 811
STEPS = 4


@pytest.mark.parametrize("precision", [sale.SALE_FP64, sale.SALE_MIXED32])
def test_largest_mesh_sod_rows_match_the_oracle(precision):
    import torch

    say("max size", N, "precision", precision)
    cfg = sale.make_config(N, N, N, t_end=1.0, precision=precision)
    r = sale.SaleRun(cfg, sale.sod_problem())
    m0, e0 = r.totals()
    r.step(STEPS)
    t, steps, _, flags = r.state()
    assert flags == 0 and steps == STEPS
    m1, e1 = r.totals()
    # the small oracle tube with the same cells along x
    g = orc.Grid(N, 4, 4, hi=(1.0, 4.0 / N, 4.0 / N), t_end=1.0)
    s = orc.sod(g)
    o = orc.Oracle(g)
    for _ in range(STEPS):
        assert o.step(s)[0] == orc.OK
    assert t == pytest.approx(s.t, rel=1e-14 if precision == sale.SALE_FP64 else 1e-6)
    tol = TOL64 if precision == sale.SALE_FP64 else 5e-6
    f = r.fields(("rho", "e", "u", "v", "w"), on_device=True)
    worst = {}
    c, w = N // 2, STEPS + 3
    for k in ("rho", "e", "u"):
        a = f[k]
        row = a[c, c]  # the middle row
        # Rows away from the walls are bitwise equal. Nodes on a wall sum
        # fewer cells and can differ from interior nodes in the last bit; that
        # rounding spreads about one row per step, so rows within STEPS + 3 of
        # a wall are held to 1e-14 instead (MIXED32: 1e-6).
        assert bool((a[w:-w, w:-w] == row).all()), f"{k}: rows away from the walls differ"
        spread = float((a - row).abs().max() / row.abs().max())
        assert spread <= (1e-14 if precision == sale.SALE_FP64 else 1e-6), (k, spread)
        ref = getattr(s, k)[1, 1]
        err = float(np.abs(row.cpu().numpy() - ref).max() / np.abs(ref).max())
        worst[k] = err
        assert err <= tol, (k, err)
    umax = float(f["u"].abs().max())
    for k in ("v", "w"):  # transverse velocity: rounding of the near-wall rows only
        assert float(f[k].abs().max()) <= (1e-14 if precision == sale.SALE_FP64 else 1e-6) * umax, k
    say("max size worst", worst, "mass", m0, m1, "energy", e0, e1)
    assert m1 == pytest.approx(m0, rel=1e-13 if precision == sale.SALE_FP64 else 1e-6)
    assert e1 == pytest.approx(e0, rel=1e-12 if precision == sale.SALE_FP64 else 1e-6)
    del f
    r.close()
    torch.cuda.empty_cache()


def test_one_past_the_largest_mesh_is_refused():
    cfg = sale.make_config(N + 1, N + 1, N + 1)
    with pytest.raises(sale.SaleError):
        sale.sale_workspace_bytes(cfg)
