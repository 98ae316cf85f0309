"""What the trained window surrogate gains over the plain solver (needs an MI355X).

The network is trained on the GPU by the library's own BF16 MFMA forward/backward kernels on
FP32 solver trajectories of the ensemble distribution (planar slopes, vegetation patches,
constant or triangular rain), then drives held-out scenarios with the water-balance gate.
Measured against the plain FP32 solver: the depth at t_end must stay within 1 % relative L1 while a
substantial share of the solver's steps is replaced by network windows; the untrained
network (the probe extrapolation alone) is run the same way for comparison.
"""
import numpy as np
import pytest

import synth
from oracle import surrogate as so
from tests.test_gpu_parity import hx  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

SIZE, T_END, K, TOL = 256, 900.0, 16, 1e-5


def test_trained_surrogate_gains_over_the_solver(hx):
    from paper_2406_14933_amd import surrogate as S
    train_sc = [synth.ensemble_member(s, size=SIZE, config=5, t_end=T_END) for s in range(8)]
    test_sc = [synth.ensemble_member(1000 + s, size=SIZE, config=5, t_end=T_END) for s in range(2)]
    window = K * 0.8 * min(S.pilot_dt(sc) for sc in train_sc[:2])
    sur = hx.Surrogate(4, 32)
    sur.set_params(so.init_params(1, 4, 32, out_scale=0.1))
    data, scales = S.collect(train_sc, list(np.linspace(window, T_END - 2 * window, 16)), window,
                             K, sur)
    losses = S.train(sur, data, 1500, batch=4, lr=1e-3, lr_end=5e-5)
    print(f"[surrogate train] window {window:.3f} s, loss {np.mean(losses[:50]):.4f} -> "
          f"{np.mean(losses[-50:]):.4f}", flush=True)
    assert np.mean(losses[-50:]) < 0.5 * np.mean(losses[:50])
    ro = S.rollout_pairs(sur, train_sc, list(np.linspace(2 * window, T_END - 2 * window, 8)),
                         window, K, scales, tol=TOL)
    S.train(sur, S.merge(data, ro), 1500, batch=4, lr=5e-4, lr_end=2e-5, seed=1)

    trained = S.evaluate(sur, test_sc, window, K, TOL)
    zero = hx.Surrogate(4, 32)
    zero.set_params(np.zeros(zero.num_params, np.float32))
    zero.set_scales(scales.as_list())
    untrained = S.evaluate(zero, test_sc, window, K, TOL)
    for name, ev in (("trained", trained), ("extrapolation only", untrained)):
        plain = sum(r["plain_steps"] for r in ev["rows"])
        solved = sum(r["surrogate_steps"] for r in ev["rows"])
        ev["avoided"] = 1.0 - solved / plain
        print(f"[surrogate {name}] err_h max {ev['err_h_max']:.2e}, accepted "
              f"{ev['accept_frac']:.2f}, solver steps avoided {ev['avoided']:.2f}, "
              f"wall {ev['surrogate_s']:.2f} s vs plain {ev['plain_s']:.2f} s", flush=True)
    # the gain is measured in solver steps avoided: the share of kept windows alone moves
    # by several points with the last-bit rounding of the FP32 trajectories it trains on
    # (0.37-0.48 trained against 0.42-0.43 untrained over builds), the steps avoided stay
    # ahead of the extrapolation's (0.36-0.41 against 0.34-0.35)
    assert trained["err_h_max"] <= 1e-2
    assert trained["avoided"] >= 0.3
    assert trained["avoided"] > untrained["avoided"]
