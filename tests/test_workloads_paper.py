"""Host checks of the paper-experiment inputs (workloads) and of the stored
table of the paper's iteration counts."""
import json
import math
import os

import numpy as np

import workloads as wl


def test_lens_model_matches_its_definition():
    # Section 4.3.1: c_min = 1/2 at x0, h = 1/(20 freq), 20-point layer outside
    for dim, freq, dofs in ((2, 40, 840), (3, 10, 240)):
        p = wl.lens_problem(dim, freq)
        assert abs(p.h - 1.0 / (20 * freq)) < 1e-15 and p.layer == 20
        assert abs(p.n[0] - dofs) <= 1  # the table's DoFs, rounded
        assert math.isclose(p.freq, freq)
        assert abs(p.c.min() - 0.5) < 1e-12 and p.c.max() <= 1.0
        i = np.unravel_index(np.argmin(p.c), p.c.shape)[::-1]  # x first
        x = [(k - p.layer) * p.h for k in i]
        x0 = (0.5, 0.1) if dim == 2 else (0.5, 0.25, 0.5)
        assert np.allclose(x, x0, atol=1e-12)
        # ten points per wavelength at c_min, and t = 0.1/freq^2 is the default
        assert math.isclose(0.5 / freq / p.h, 10.0)
        assert math.isclose(p.default_t(), 0.1 / freq ** 2)
        f = wl.lens_source(p)
        (k,) = np.flatnonzero(f)
        assert np.allclose([(c - p.layer) * p.h for c in np.unravel_index(k, f.shape)], 0.5)


def test_homogeneous_model_and_dipole_source():
    p = wl.homog_problem(2, 40)
    assert p.n == (421, 421) and abs(p.h - 1 / 400) < 1e-15 and p.layer == 10
    assert math.isclose(p.default_t(), 0.4 / 40 ** 2)
    f = wl.dipole_source(p).real
    # zero net charge; the positive lobe 6h right of the centre, the negative left
    assert abs(f.sum()) * p.h ** 2 < 1e-12
    assert np.unravel_index(np.argmax(f), f.shape) == (210, 216)
    assert np.unravel_index(np.argmin(f), f.shape) == (210, 204)
    # each lobe is a normalised Gaussian: the positive one alone integrates to one
    lobe = wl.gaussian_source(p, (0.5 + p.layer * p.h + 6 * p.h, 0.5 + p.layer * p.h), 3 * p.h).real
    assert math.isclose(lobe.sum() * p.h ** 2, 1.0, rel_tol=1e-9)
    assert np.allclose(f, lobe - np.roll(lobe, -12, axis=1), atol=1e-9 * lobe.max())
    q = wl.homog_problem(3, 10)
    g = wl.dipole_source(q).real
    assert q.n == (121, 121, 121) and abs(g.sum()) * q.h ** 3 < 1e-12
    c = 60
    for ax in range(3):  # a pair along every axis
        hi = [c, c, c]
        lo = [c, c, c]
        hi[2 - ax] += 6
        lo[2 - ax] -= 6
        assert g[tuple(hi)] > 0 > g[tuple(lo)]


def test_stored_paper_tables_are_well_formed():
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")))
    assert len(d["shift_2d"]["rows"]) == 16 and len(d["fprtol_3d"]["rows"]) == 12 and len(d["lens"]["rows"]) == 6
    assert [len(r["inner"]) for r in d["noshift_2d"]["rows"]] == [3, 4, 4, 4]
    for key in ("shift_2d", "fprtol_3d", "lens"):
        assert d[key]["citation"].startswith("Section 4.")
        for r in d[key]["rows"]:
            assert r["outer"] >= 1 and r["inner"] >= 1.0 and r["std"] >= 0.0
