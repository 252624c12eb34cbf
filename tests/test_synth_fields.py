"""Seeded generators: determinism, valid compositions and the class mix of
the detonation patch."""
import numpy as np

from synth import fields


def test_c1_seeded_and_valid():
    a, b = fields.c1_cells(256), fields.c1_cells(256)
    assert np.array_equal(a.Y, b.Y) and np.array_equal(a.T, b.T)
    assert np.all(a.Y >= 0) and np.allclose(a.Y.sum(0), 1.0, atol=1e-14)
    assert a.T.min() >= 1000 and a.T.max() <= 2500
    assert a.p.min() >= 101325 and a.p.max() <= 20 * 101325


def test_c2_class_fractions():
    c = fields.c2_field(256, 64, 8)
    frac = np.bincount(c.cls, minlength=3) / c.cls.size
    assert abs(frac[0] - 0.85) < 0.02 and abs(frac[1] - 0.05) < 0.01 and abs(frac[2] - 0.10) < 0.02
    cold = c.cls == 0
    assert np.all(c.T[cold] == 300.0)
    assert np.all((c.T[c.cls == 1] > 1400) & (c.T[c.cls == 1] < 3200))
    assert np.allclose(c.Y.sum(0), 1.0, atol=1e-14)
    # x fastest: id = x + nx (y + ny z); the front moves along +x, burnt gas at small x
    assert c.cls[0] == 2 and c.cls[255] == 0


def test_c3_box_mix():
    boxes = fields.c3_boxes()
    assert len(boxes) == 400
    tot = sum(int(np.prod(b.shape)) for b in boxes)
    assert 5.7e6 <= tot <= 6.3e6
    assert {b.level for b in boxes} == {0, 1, 2}
    s = fields.c3_box_state(boxes[5], box_id=5)
    assert np.allclose(s.Y.sum(0), 1.0, atol=1e-14) and s.T.min() >= 290 and s.T.max() <= 2900


def test_eq_table_reproduces_grid_points():
    tab = fields.eq_table("m9_eq_ZTp.npz")
    Y = tab(Z=tab.axes[0][3], T=tab.axes[1][7], lnp=tab.axes[2][2])
    assert np.allclose(Y[:, 0], tab.Y[3, 7, 2], rtol=0, atol=1e-16)
