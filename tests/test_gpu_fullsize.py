"""Parity at full size, in the launch configuration the benchmark times:
the D=12 precision workload (646,646 coefficients, 17 grids, 3.5e9
samples).  Sampled outputs the oracle computes one by one: function values
at random nodes of every grid, and DCT-I entries of the gathered right-hand
side b for random rows of the two smallest grids (each entry by its
definition, a full-grid sum of samples times products of DCT-I rows)."""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(
    not os.path.exists(os.path.join(os.path.dirname(__file__), "golden", "cfg4_meta.json")),
    reason="oracle reference data not generated yet")]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup():
    from paper_2309_14584_amd import fct
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    torch.cuda.set_device(0)
    with open(os.path.join(os.path.dirname(__file__), "golden", "cfg4_meta.json")) as fh:
        meta = json.load(fh)
    prob = W.config4(min_grids=meta["K"])
    plan = fct.Plan(prob.support, prob.grids)
    samples = plan.sample(prob.family, prob.params)
    yield fct, prob, plan, samples
    plan.close()


def test_samples_at_random_nodes(setup):
    fct, prob, plan, samples = setup
    rng = np.random.default_rng(71)
    offs = np.concatenate([[0], np.cumsum(prob.points)])
    for l in range(prob.K):
        idx = rng.integers(0, prob.points[l], size=120)
        got = samples[torch.as_tensor(offs[l] + idx, device="cuda")].cpu().numpy()
        X = np.concatenate([O.grid_coordinates(prob.grids[l], int(k), int(k) + 1) for k in idx])
        ref = O.function_values(prob.family, prob.params, X)
        assert np.max(np.abs(got - ref)) <= 1e-14, l


@pytest.fixture(scope="module")
def entries(setup):
    """Oracle DCT-I entries of 5 random rows of each of the two smallest grids."""
    fct, prob, plan, samples = setup
    rng = np.random.default_rng(73)
    out = []
    for l in np.argsort(prob.points)[:2]:
        g = prob.grids[l]
        bins = np.unique(O.alias_bins(prob.support, g))        # the grid's rows, in row order
        pick = rng.choice(len(bins), size=5, replace=False)
        multis = np.stack(np.unravel_index(bins[pick], tuple(int(N) + 1 for N in g)), axis=1)
        ref, scale = O.dct_entries(prob.family, prob.params, g, multis)
        out.append((int(l), len(bins), pick, ref, scale))
    return out


@pytest.mark.parametrize("mode", ["vector", "matrix"])
def test_dct_entries_of_the_smallest_grids(setup, entries, mode):
    fct, prob, plan, samples = setup
    plan.set_dct_engine(fct.DCT_F64, fct.ENGINE_MATRIX if mode == "matrix"
                        else fct.ENGINE_VECTOR)
    b = plan.dct(samples).cpu().numpy()
    plan.set_dct_engine(fct.DCT_F64, fct.ENGINE_VECTOR)
    for l, nrows, pick, ref, scale in entries:
        points, rows, p_off, r_off = plan.grid(l)
        assert rows == nrows
        err = np.abs(b[r_off + pick] - ref) / scale
        print(f"{mode}: grid {l} ({points} points): max error / abs-sum {err.max():.2e}")
        assert np.all(err <= 1e-13)
