"""GPU test of the surrogate-pruned search (reduced sizes): labels from the
batched GBD sweep, training on the device, top-32 proposals re-scored by
plain GBD, compared with the exhaustive sweep of the same candidate pool, with
random orders and draws of candidates, and with a model-free heuristic."""
import numpy as np
import pytest

from paper_2404_12454_amd import surrogate
from gbd_testutil import ensure_library

pytestmark = pytest.mark.gpu


def test_surrogate_prunes_the_search():
    """231 candidates (OF 11 x q 7 x 48, 96, 128 across) at 128 x 128 over
    +-8 lambda F; 11 of them lie within 1 % of the exhaustive optimum (at 96
    across: the figure of merit is not monotone in the count).  Taken in the
    network's order, GBD meets one of them within 3 re-scores, before the
    median of 101 random orders and before the heuristic (most beamlets,
    OF q nearest 1.7); the top 32 land within 0.5 % of the optimum and do no
    worse than the median of 5 random draws of 32."""
    ensure_library()
    pool = surrogate.candidate_pool(n_of=11, n_q=7, nacross=(48, 96, 128))
    rec = surrogate.run(n_train=3000, epochs=60, pool=pool, top=32, label_npix=128, rescore_npix=128, span=8.0,
                        random_baselines=5, random_orders=101, within=1.01)
    print({k: v for k, v in rec.items() if k != "loss_history"}, flush=True)
    assert rec["val_r2"] > 0.99
    assert rec["rescores_to_reach_surrogate"] <= 3
    assert rec["rescores_to_reach_surrogate"] < rec["rescores_to_reach_random_median"]
    assert rec["rescores_to_reach_surrogate"] < rec["rescores_to_reach_heuristic"]
    assert rec["rms_ratio_to_optimum"] <= 1.005
    assert rec["rms_ratio_to_optimum"] <= float(np.median(rec["random32_ratio_to_optimum"]))
    assert rec["rms_ratio_to_optimum"] < rec["heuristic32_ratio_to_optimum"]
    # No timing assertion at this size: the exhaustive sweep over 231 small
    # instances is one call of ~50 ms and the online phase (inference, then one
    # 32-instance call) ~2 calls, so their ratio is set by per-call costs that
    # vary between runs (below 1 in one run, above 1 in others).  The full-size
    # test below asserts the speed-up where the sweep is what costs (8,897
    # candidates at 512 x 512).


def test_surrogate_full_size_finds_the_optimum_first():
    """The full-size search: 20,000 labels at 256 x 256, 200 epochs, the
    8,897-candidate pool re-scored at 512 x 512 over +-8 lambda F.  207
    candidates lie within 1 % of the optimum (all at 96 across); taken in the
    network's order, GBD meets one within 3 re-scores, before the median of
    101 random orders and before the heuristic order; the top 32 contain a
    candidate with the optimum's RMS (the same OF q); the online phase is at
    least 50 times faster than the exhaustive sweep."""
    ensure_library()
    rec = surrogate.run(random_baselines=5, random_orders=101)
    print({k: v for k, v in rec.items() if k != "loss_history"}, flush=True)
    assert rec["val_r2"] > 0.999
    assert rec["candidates_within"] > 100
    assert rec["rescores_to_reach_surrogate"] <= 3
    assert rec["rescores_to_reach_surrogate"] < rec["rescores_to_reach_random_median"]
    assert rec["rescores_to_reach_surrogate"] < rec["rescores_to_reach_heuristic"]
    assert rec["rms_ratio_to_optimum"] <= 1.0 + 1e-9
    assert rec["rms_ratio_to_optimum"] <= min(rec["random32_ratio_to_optimum"])
    assert rec["speedup_online"] > 50


def test_surrogate_is_flat_in_fnumber_and_wavelength():
    """In lambda*F units the figure of merit does not depend on F# or lambda;
    the trained network's predictions must vary little along them."""
    import paper_2404_12454_amd as gbd
    ctx = gbd.Context(0)
    from paper_2404_12454_amd import scenes
    draws = scenes.surrogate_draws(3000, 7)
    y = np.log10(surrogate.score(ctx, draws, 128, 8.0)[:, 0])
    sur = surrogate.Surrogate(ctx).fit(draws, y, epochs=60, init_params=surrogate.init_params(seed=0))
    base = np.array([1.6, 1.0, 48, 10.0, 1e-6])
    grid = []
    for fn in np.linspace(4, 20, 9):
        for lam in np.exp(np.linspace(np.log(0.4e-6), np.log(2e-6), 9)):
            grid.append([base[0], base[1], base[2], fn, lam])
    p = sur.predict(np.array(grid))
    spread = p.max() - p.min()
    print("spread along F#, lambda:", spread, "label range:", np.ptp(y), flush=True)
    assert spread < 0.15 * np.ptp(y)
