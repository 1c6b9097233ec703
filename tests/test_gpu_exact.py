"""Exact reference mode on the GPU: every pair through the exact Galerkin
integral of eq. "matrix" (closed forms of section 3.4's integrals, or the
semi-analytic route where the corner sum would lose digits), selected by a
near_eta larger than any separation/diameter ratio of the layout.

Bars: entries 1e-10 relative against the oracle's high-accuracy entries
(exact integrals within 4 diameters, 8 x 8 Gauss beyond, whose error there is
below 1e-13); capacitances 1e-9 against the oracle's extraction with the same
rule.  All pairs must be on the exact path: n_near = N (N + 1) / 2.
"""
import sys

import numpy as np
import pytest

import gbem_inputs as gi
import oracle
from paper_2203_11733_amd import binding

pytestmark = pytest.mark.gpu
EXACT_ETA = 1e6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = binding.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("layout", [gi.crossing_bars_in_box(), gi.random_small_layout(2)],
                         ids=["bars_in_box", "random2"])
def test_exact_mode_entries(ctx, layout):
    lo, hi, cond = binding.mesh_layout(layout)
    n = lo.shape[0]
    rng = np.random.default_rng(11)
    ii = rng.integers(0, n, 3000).astype(np.int32)
    jj = rng.integers(0, n, 3000).astype(np.int32)
    got = ctx.assemble_sample(lo, hi, ii, jj, binding.make_opts(3, EXACT_ETA))
    ref = oracle.entries(lo, hi, ii, jj, 8, 4.0)
    err = np.abs(got - ref) / np.abs(ref)
    say(f"exact mode {layout.name} N={n}: max rel entry err {err.max():.3e}")
    assert err.max() < 1e-10


@pytest.mark.parametrize("layout", [gi.two_plates(), gi.crossing_bars_in_box()], ids=["two_plates", "bars_in_box"])
def test_exact_mode_capacitance(ctx, layout):
    lo, hi, cond = binding.mesh_layout(layout)
    n, m = lo.shape[0], layout.n_conductors
    C, rep = ctx.extract(lo, hi, cond, m, layout.eps_r, layout.length_unit_m, binding.make_opts(3, EXACT_ETA))
    assert rep["n_near"] == n * (n + 1) // 2
    Co = oracle.extract_panels(lo, hi, cond, m, layout.eps_r, layout.length_unit_m, 8, 4.0)
    rel = float(np.abs(C - Co).max() / np.abs(Co).max())
    say(f"exact mode {layout.name}: C rel vs oracle (p=8, eta=4) {rel:.2e}")
    assert rel < 1e-9
