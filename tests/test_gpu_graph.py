"""Graph replay of an extraction's launch sequence (opts.graph): the same
kernels as direct launches, so the capacitances must be identical, bit for
bit, on first instantiation, on updates of a cached executable by a new
capture of the same topology, with direct-launch work between replays, and
for jobs run concurrently by the serving loop."""
import sys

import numpy as np
import pytest

import gbem_inputs as gi
from paper_2203_11733_amd import binding

pytestmark = pytest.mark.gpu

MODES = {
    "f64": dict(),
    "mixed": dict(far_dtype="f32", factor_dtype="f16", refine_tol=1e-8, max_refine=40),
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def meshes(gpu_lib):
    # three sizes, two of them in the same padded order (an update of the
    # cached executable), one in another (an instantiation)
    out = []
    for seed, target in ((3, 1500), (5, 1500), (9, 2600)):
        rng = np.random.default_rng(seed)
        for _ in range(200):
            lay = gi.random_manhattan(rng, n_target=target)
            lo, hi, cond = binding.mesh_layout(lay)
            if abs(lo.shape[0] - target) <= 0.25 * target:
                break
        out.append((lay, lo, hi, cond))
    return out


@pytest.mark.parametrize("mode", sorted(MODES))
def test_graph_replay_equals_direct_launches(meshes, mode):
    o_direct = binding.make_opts(3, 2.0, **MODES[mode])
    o_graph = binding.make_opts(3, 2.0, graph=True, **MODES[mode])
    with binding.Context(0) as ctx:
        ref = []
        for lay, lo, hi, cond in meshes:
            C, rep = ctx.extract(lo, hi, cond, lay.n_conductors, lay.eps_r, lay.length_unit_m, o_direct)
            assert rep["graph_used"] == 0
            ref.append(C)
        # graph calls interleaved with direct ones, every mesh twice
        order = [0, 1, 2, 0, 1, 2]
        for step, k in enumerate(order):
            lay, lo, hi, cond = meshes[k]
            C, rep = ctx.extract(lo, hi, cond, lay.n_conductors, lay.eps_r, lay.length_unit_m, o_graph)
            npad = -(-lo.shape[0] // 512) * 512
            say(f"{mode} step {step}: N={lo.shape[0]} npad={npad} graph_used={rep['graph_used']}"
                f" instantiated={rep['graph_instantiated']} refine={rep['refine_iters']}"
                f" max|dC|={np.abs(C - ref[k]).max():.1e}")
            assert rep["graph_used"] == 1
            # the second pass over a mesh finds its executable cached: an update
            # by the new capture (new flags epochs and tickets), no instantiation
            if step >= 3:
                assert rep["graph_instantiated"] == 0
            assert np.array_equal(C, ref[k])
            # direct launches between replays
            lay2, lo2, hi2, cond2 = meshes[(k + 1) % len(meshes)]
            C2, _ = ctx.extract(lo2, hi2, cond2, lay2.n_conductors, lay2.eps_r, lay2.length_unit_m, o_direct)
            assert np.array_equal(C2, ref[(k + 1) % len(meshes)])


@pytest.mark.parametrize("mode", sorted(MODES))
def test_served_graph_jobs_equal_direct(meshes, mode):
    """Jobs submitted with opts.graph run four at a time in the serving loop
    (each worker with its own cached executables) and match direct launches."""
    o_direct = binding.make_opts(3, 2.0, **MODES[mode])
    o_graph = binding.make_opts(3, 2.0, graph=True, **MODES[mode])
    with binding.Context(0) as ctx:
        ref = [ctx.extract(lo, hi, cond, lay.n_conductors, lay.eps_r, lay.length_unit_m, o_direct)[0]
               for lay, lo, hi, cond in meshes]
        jobs = [ctx.submit(lo, hi, cond, lay.n_conductors, lay.eps_r, lay.length_unit_m, o_graph)
                for _ in range(3) for lay, lo, hi, cond in meshes]
        results = [j.wait(120.0) for j in jobs]
        for j in jobs:
            j.free()
    used = sum(rep["graph_used"] for _, rep in results)
    say(f"served {mode}: {len(results)} jobs, {used} as graphs")
    assert used == len(results)
    for i, (C, rep) in enumerate(results):
        assert np.array_equal(C, ref[i % len(meshes)])


@pytest.mark.parametrize("mode", sorted(MODES))
def test_graph_after_workspace_growth(meshes, mode):
    """A larger job between two graph runs of the same shape grows the
    workspace (new buffer addresses): the second run gets a new executable
    rather than an update of the old one, and the results stay exact."""
    o_direct = binding.make_opts(3, 2.0, **MODES[mode])
    o_graph = binding.make_opts(3, 2.0, graph=True, **MODES[mode])
    small, big = meshes[0], meshes[2]
    with binding.Context(0) as ctx:
        ref = ctx.extract(*small[1:], small[0].n_conductors, small[0].eps_r, small[0].length_unit_m, o_direct)[0]
    with binding.Context(0) as ctx:
        runs = []
        for lay, lo, hi, cond in (small, big, small, small):
            runs.append(ctx.extract(lo, hi, cond, lay.n_conductors, lay.eps_r, lay.length_unit_m, o_graph))
    say(f"{mode}: instantiated {[r[1]['graph_instantiated'] for r in runs]}")
    assert all(r[1]["graph_used"] == 1 for r in runs)
    assert [r[1]["graph_instantiated"] for r in runs] == [1, 1, 1, 0]
    for k in (0, 2, 3):
        assert np.array_equal(runs[k][0], ref)
