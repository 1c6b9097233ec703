"""GPU tests of the multi-dielectric path (section 4) against the oracle.

The library integrates the double-layer kernel over near pairs in closed form
and over far pairs with the closed-form inner integral under an n x n Gauss
rule on the target, n from 6 at the near threshold eta = 2 down to 2 at 40
diameters (each within about 1e-13 |I_i| of the exact value); the oracle
integrates the target adaptively to 1e-12.  So Q entries agree to 1e-12 |I_i| (Q_ik is at most |I_i| / 2 in
size), and capacitances with the same single-layer rule on both sides (exact
near pairs, 3 x 3 Gauss far pairs) to 1e-11 of max |C| (the solves: a direct
LU in the oracle, the normal equations refined to a residual of 1e-13 on the
GPU; measured differences are about 1e-14).  At the larger size the checks are
properties that hold at any size: Gauss's theorem on every wire's closed
surface, the layout's mirror symmetry, the signs of a Maxwell matrix.
"""
import sys

import numpy as np
import pytest

import gbem_inputs as gi
from oracle import dielectric as od
from oracle import dielectric_partition as odp
from paper_2203_11733_amd import binding

pytestmark = pytest.mark.gpu

Q_TOL = 1e-12         # |Q_gpu - Q_oracle| / |I_i|
C_TOL = 1e-11         # |C_gpu - C_oracle| / max |C_oracle|


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = binding.Context(0)
    yield c
    c.close()


def _areas(m):
    e = m.hi - m.lo
    return np.prod(np.where(e == 0, 1.0, e), axis=1)


def _wire_members(m):
    """Panel indices of each net and the outward sign (+1 where the wire's
    outward normal is + along the panel's axis: the dielectric on the + side)."""
    out = []
    for c in range(m.n_conductors):
        idx = np.flatnonzero((m.kind == gi.CONDUCTOR) & (m.conductor == c))
        out.append((idx, np.where(m.region_plus[idx] >= 0, 1.0, -1.0)))
    return out


def test_double_layer_entries_vs_oracle(ctx):
    """Sampled Q_ik of a 404-panel stack (near pairs of every orientation,
    far pairs, coplanar pairs) against the oracle's adaptive integral."""
    m = gi.layered_stack(3, 0.5)
    say(f"double layer: {m.name} n={m.n_panels}")
    Q = ctx.assemble_double_layer(m.lo, m.hi, 2.0)
    area = _areas(m)
    rng = np.random.default_rng(7)
    n = m.n_panels
    # pairs close to each other (where the rule is hardest) and random ones
    cen = 0.5 * (m.lo + m.hi)
    d = np.sqrt(((cen[:, None, :] - cen[None, :, :]) ** 2).sum(-1))
    near = np.argwhere((d < 0.6) & ~np.eye(n, dtype=bool))
    pick = near[rng.choice(len(near), 150, replace=False)]
    pick = np.vstack([pick, rng.integers(0, n, size=(100, 2))])
    worst = 0.0
    for i, k in pick:
        ref = od.double_layer_pair(m.lo[i], m.hi[i], m.lo[k], m.hi[k])
        err = abs(Q[i, k] - ref) / area[i]
        worst = max(worst, err)
        assert err <= Q_TOL, (i, k, Q[i, k], ref)
        if ref == 0.0:
            assert Q[i, k] == 0.0
    say(f"  {len(pick)} sampled entries: max |dQ| / |I_i| = {worst:.2e}")
    assert np.all(np.diag(Q) == 0.0)


def test_double_layer_gauss_theorem(ctx):
    """Sum over a closed wire surface of the outward double layer is -|I_i|/2
    for a panel on it and 0 for a panel outside (at a bench-sized stack)."""
    m = gi.layered_stack(3, 0.15)
    say(f"gauss theorem: {m.name} n={m.n_panels}")
    Q = ctx.assemble_double_layer(m.lo, m.hi, 2.0)
    area = _areas(m)
    worst_on = worst_off = 0.0
    for idx, sgn in _wire_members(m):
        s = Q[:, idx] @ sgn
        on = np.zeros(m.n_panels, bool)
        on[idx] = True
        e_on = np.abs(s[on] + 0.5 * area[on]) / area[on]
        e_off = np.abs(s[~on]) / area[~on]
        worst_on, worst_off = max(worst_on, e_on.max()), max(worst_off, e_off.max())
    say(f"  on the surface {worst_on:.2e}, off it {worst_off:.2e} (relative to |I_i|)")
    assert worst_on <= 1e-11 and worst_off <= 1e-11


def test_two_slab_vs_oracle_and_closed_form(ctx):
    """Two dielectric slabs between plates: GPU C against the oracle at 4 x 2
    panels per face, then toward eps0 L^2 / (d1/eps1 + d2/eps2) as the
    mesh is refined."""
    m = gi.two_slab_capacitor(n_xy=4, n_z=2)
    say(f"two slab: {m.name} n={m.n_panels}")
    C, rep = ctx.extract_dielectric(*m.args())
    ref = od.extract(*m.args(), single_layer=(3, 2.0))
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    say(f"  C vs oracle {err:.2e}, residual {rep['residual']:.1e}, sweeps {rep['refine_iters']}")
    assert err <= C_TOL
    assert rep["residual"] <= 1e-12
    L, d1, d2, e = 1.0, 0.3, 0.7, [4.0, 1.0]
    exact = gi.EPS0 * 1e-6 * L * L / (d1 / e[0] + d2 / e[1])
    errs = []
    for nxy, nz in ((4, 2), (8, 4), (16, 8)):
        C, _ = ctx.extract_dielectric(*gi.two_slab_capacitor(L, d1, d2, nxy, nz, e).args())
        errs.append(C[0, 0] / exact - 1.0)
        assert C[0, 0] > 0 and C[1, 0] < 0
    say(f"  C00 / exact - 1 at 4, 8, 16 panels across: {errs}")
    assert errs[0] > errs[1] > errs[2] > 0 and errs[2] < 0.03


def test_layered_stack_vs_oracle(ctx):
    """Two wires in a three-layer stack (grounded top and bottom, Neumann
    walls, two interfaces), 132 panels: GPU C against the oracle."""
    m = gi.layered_stack(1, 0.5)
    say(f"layered stack: {m.name} n={m.n_panels}")
    C, rep = ctx.extract_dielectric(*m.args())
    ref = od.extract(*m.args(), single_layer=(3, 2.0))
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    say(f"  C vs oracle {err:.2e}, residual {rep['residual']:.1e}")
    assert err <= C_TOL


def test_three_region_triangle_vs_oracle(ctx):
    """A third dielectric embedded under the interface of the two-slab
    capacitor: every region borders both others, so the unknowns of one
    region do not form one contiguous slot range (the blocked M^T M covers a
    range with other regions' unknowns inside); 124 panels against the
    oracle."""
    m = gi.two_slab_with_block()
    say(f"three regions: {m.name} n={m.n_panels}")
    C, rep = ctx.extract_dielectric(*m.args())
    ref = od.extract(*m.args(), single_layer=(3, 2.0))
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    say(f"  C vs oracle {err:.2e}, residual {rep['residual']:.1e}")
    assert err <= C_TOL


def test_single_region_grounded_box(ctx):
    """One dielectric inside a grounded box (conductor and Dirichlet panels
    only: the section 4 system then holds the direct form of the section 3
    problem). GPU against the oracle at 116 panels; and the finer direct
    solution against the library's single-dielectric (indirect, section 3)
    extraction of the same geometry: both approximate the same capacitances,
    within 1 % here (observed 0.1 %; the two discretisations differ)."""
    m = gi.bars_in_grounded_box()
    say(f"grounded box: {m.name} n={m.n_panels}")
    C, rep = ctx.extract_dielectric(*m.args())
    ref = od.extract(*m.args(), single_layer=(3, 2.0))
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    say(f"  C vs oracle {err:.2e}")
    assert err <= C_TOL
    fine = gi.bars_in_grounded_box(0.5, 1.0)
    Cd, _ = ctx.extract_dielectric(*fine.args())
    lay = gi.bars_in_grounded_box_layout(0.5)
    Cs, _ = ctx.extract_layout(lay)
    dev = float(np.abs(Cd - Cs).max() / np.abs(Cs).max())
    say(f"  direct ({fine.n_panels} panels) vs single-dielectric: {Cd.ravel() / 1e-18} vs {Cs.ravel() / 1e-18} aF,"
        f" max deviation {dev:.3f}")
    assert dev <= 0.01
    assert np.all(np.diag(Cd) > 0) and Cd[0, 1] < 0


def test_partitioned_layout_vs_oracle(ctx):
    """One mesh per main net by the section 3.3 / 4.1 rules (the paper's
    method for several dielectrics): meshes and every column of C against the
    oracle's mesher and extraction."""
    lay = gi.layered_stack_layout(1)
    rule = (0.5, 2.0, 1.0, 0.5)
    C, panels, rep = ctx.extract_dielectric_partitioned(lay, *rule)
    ref, ref_panels = odp.extract(lay, *rule)
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    say(f"partitioned: panels {list(panels)}, C vs oracle {err:.2e}")
    assert list(panels) == ref_panels
    assert err <= C_TOL


def test_partitioned_lanes_equal_single_extractions(ctx):
    """The per-main-net extractions run concurrently on up to four lanes
    (own workspace and stream each); every column equals, bit for bit, the
    synchronous entry's extraction of that net's mesh."""
    lay = gi.layered_stack_layout(3)
    rule = (0.25, 2.0, 1.0, 0.5)
    C, panels, rep = ctx.extract_dielectric_partitioned(lay, *rule)
    for k in range(lay.n_conductors):
        lo, hi, kind, cond, rp, rm = binding.mesh_dielectric_partition(lay, k, *rule)
        assert lo.shape[0] == panels[k]
        Ck, _ = ctx.extract_dielectric(lo, hi, kind, cond, rp, rm, lay.eps_r, lay.n_conductors, lay.length_unit_m)
        assert np.array_equal(C[:, k], Ck[:, k]), k
    C2, _, _ = ctx.extract_dielectric_partitioned(lay, *rule)
    assert np.array_equal(C, C2)
    say(f"partitioned lanes: {lay.n_conductors} columns equal the single extractions")


def test_partitioned_layout_accuracy(ctx):
    """The per-main-net meshes of the six-net stack against its uniform
    8,644-panel mesh: the same capacitances to discretisation accuracy with a
    fraction of the panels (the point of the paper's partition)."""
    lay = gi.layered_stack_layout(3)
    C, panels, rep = ctx.extract_dielectric_partitioned(lay, 0.04, 4.0, 0.5, 0.5)
    fine = gi.layered_stack(3, 0.1)
    Cf, _ = ctx.extract_dielectric(*fine.args())
    dev = float(np.max(np.abs(np.diag(C) - np.diag(Cf)) / np.diag(Cf)))
    cdev = float(np.abs(C - Cf).max() / np.abs(Cf).max())
    say(f"partitioned: panels {list(panels)} against {fine.n_panels}; diagonal within {dev:.4f},"
        f" whole matrix within {cdev:.4f} of max |C|, {rep['t_total_ms']:.1f} ms for all six meshes")
    say(f"  diag partitioned {np.diag(C) / 1e-18} aF, uniform {np.diag(Cf) / 1e-18} aF")
    assert max(panels) * 3 < fine.n_panels
    assert dev <= 0.02 and cdev <= 0.02


def test_exact_single_layer_mode(ctx):
    """near_eta = 1e6 puts every single-layer pair on the exact path (the
    exact reference mode); the double layer keeps its own split at eta = 2
    (its closed form loses digits with distance).  Against the oracle with
    the exact G_ij for every pair."""
    m = gi.layered_stack(1, 0.5)
    o = binding.make_opts(3, 1e6)
    C, rep = ctx.extract_dielectric(*m.args(), opts=o)
    ref = od.extract(*m.args())
    err = float(np.abs(C - ref).max() / np.abs(ref).max())
    say(f"exact single layer: near pairs {rep['n_near']} of {m.n_panels * (m.n_panels + 1) // 2}, C vs oracle {err:.2e}")
    assert rep["n_near"] == m.n_panels * (m.n_panels + 1) // 2
    assert err <= C_TOL


def test_layered_stack_properties_at_size(ctx):
    """Six wires, 4,368 panels: the mirror y -> W - y maps wire 0 to wire 2
    and each upper wire to itself, so C is invariant under that exchange;
    a Maxwell matrix has C_kk > 0 and C_nk < 0 off the diagonal."""
    m = gi.layered_stack(3, 0.15)
    say(f"layered stack: {m.name} n={m.n_panels}")
    C, rep = ctx.extract_dielectric(*m.args())
    say(f"  residual {rep['residual']:.1e} after {rep['refine_iters']} sweeps, asym {rep['asym']:.2e},"
        f" {rep['t_total_ms']:.1f} ms")
    perm = [2, 1, 0, 3, 4, 5]
    P = C[np.ix_(perm, perm)]
    assert float(np.abs(P - C).max() / np.abs(C).max()) <= 1e-9
    assert np.all(np.diag(C) > 0)
    assert np.all(C[~np.eye(6, dtype=bool)] < 0)
    assert rep["residual"] <= 1e-12


def test_dielectric_rejects_inconsistent_mesh(ctx):
    m = gi.two_slab_capacitor(n_xy=2, n_z=1)
    rm = m.region_minus.copy()
    rm[0] = m.region_plus[0] if m.region_plus[0] >= 0 else 0   # conductor panel with two sides
    args = list(m.args())
    args[5] = rm
    with pytest.raises(binding.GbemError, match="panel 0"):
        ctx.extract_dielectric(*args)
