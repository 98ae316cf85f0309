"""Shared test helpers: run a synth scenario through the oracle or the HIP library."""
import numpy as np

import oracle


def ref_grid(sc):
    return oracle.grid(sc.nq, sc.nr, sc.a, sc.side, sc.segs, sc.active, sc.mask_code)


def ref_params(sc):
    return oracle.params(sc.g, sc.cfl, sc.dt_max, sc.h_dry, sc.alpha_s, sc.tau_lin, sc.visc,
                         sc.f_inf, sc.h_inf)


def ref_rain(sc):
    return oracle.rain(sc.rain_kind, sc.i_a, sc.t_a, sc.T_d)


def ref_run(sc, t_end=None, max_steps=10 ** 9, nthreads=0, log_dt=False):
    G = ref_grid(sc)
    h, v1, v2, b, dl = oracle.run(G, sc.z, sc.theta, sc.alpha_p, ref_params(sc), ref_rain(sc),
                                  sc.h0, sc.v10, sc.v20, sc.t_end if t_end is None else t_end,
                                  max_steps=max_steps, nthreads=nthreads, log_dt=log_dt)
    th = np.where(G.active | G.dirichlet, sc.theta, np.where(G.flux, 1.0, 0.0))
    return {"h": h, "v1": v1, "v2": v2, "q1": th * h * v1, "q2": th * h * v2,
            "books": b.as_dict(), "dt": dl}


def rel_l1(a, b):
    den = np.abs(b).sum()
    return np.abs(a - b).sum() / (den if den > 0 else 1.0)
