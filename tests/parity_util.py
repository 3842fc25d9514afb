"""Lockstep trajectory parity between the oracle and the GPU integrator
(shared by the GPU test modules; not collected as tests)."""
import numpy as np


def wrms_diff(a, b, rtol, atol):
    w = 1.0 / (rtol * np.abs(b) + atol)
    return float(np.sqrt(np.mean(((a - b) * w) ** 2)))


def cell_wrms(a, b, rtol, atol, n):
    """Per-cell WRMS difference (uniform cell size n)."""
    w = 1.0 / (rtol * np.abs(b) + atol)
    return np.sqrt(np.mean((((a - b) * w) ** 2).reshape(-1, n), 1))


def gpu_bdf(G, prob, dev, **kw):
    return G.Bdf.from_problem(prob, device=dev, **kw)


# Bars of the lockstep trajectory comparison (compare_trajectory).
# While every decision agrees the two sides' states still differ: the
# Newton iteration stops once its correction is 0.1 of the tolerance, and
# the rounding of those unconverged iterates (the GPU's FMA and tree sums,
# the oracle's serial sums without contraction; stiff components scale it
# by gamma J) differs by up to ~6e-6 WRMS per step on the random networks
# (measured: 1.3e-3 after 2,560 steps of 256 10-species cells, 5.8e-3 after
# 960 steps of the 4,096-unknown uneven batch; 1.5e-6 after the 3,778
# steps of the Robertson run).  States at a common time must agree within
# END_BAR0 + END_BAR_PER_STEP * (steps taken).
END_BAR0 = 1e-3
END_BAR_PER_STEP = 2e-5
# With the lazy Newton matrix the convergence-rate estimate carries over
# between attempts, so the grouped test (WRMS over all cells) accepts a
# first correction of up to 0.1 / crate: single cells may stop well short
# of convergence, and the rounding of their unconverged states then shows
# at up to ~4e-5 WRMS per step over the 256-cell network (measured: 0.079
# after 1,984 steps; 0.049 after 2,176 with variable coefficients).
END_BAR_PER_STEP_LAZY = 1e-4
# The step sizes drift apart through the same rounding: each change of h
# multiplies it by eta = (1.2 err)^(-1/(q+1)), err being the WRMS norm of
# acor = y_n - z0[0], a difference of two states that agree to about the
# tolerance.  Measured: 3.7e-9 over the Robertson run, 8e-7 after 2,300
# steps of the 256-cell network, and it can grow to a few percent late in
# runs where small components (weighted by 1/atol) dominate err.  Once it
# passes FLIP_H the two runs take materially different steps (their states
# then differ by a fraction of the tolerance: 0.07-0.09 WRMS measured after
# 1,400-3,300 steps), which is judged like a flipped decision; a decision
# taken differently at a threshold changes h by at least the 1.5x of the
# hysteresis, or the attempt count for a failed test.
FLIP_H = 1e-3
# After a decision flip both runs are valid integrations at the same
# tolerance: the GPU's error against a tight-tolerance oracle run must be
# within this factor of the oracle's own error against it.
FLIP_ERR_RATIO = 3.0

_REF_CACHE = {}


def _decisions(sg, so):
    """(attempts, Newton iterations, order, Newton-matrix setups, attempts
    redone with fresh factors, GMRES iterations) of both sides after a
    step."""
    keys = ("nattempts", "nniters", "q", "nsetups", "nstale_retries", "nliters")
    return tuple(sg[k] for k in keys), tuple(so[k] for k in keys)


def gpu_y_at(gb, t):
    """The GPU solution at time t near its current time, from its Nordsieck
    history: y(t_n + s h) = sum_j z[j] s^j (the step sizes of the two sides
    differ by rounding, so after the same number of steps their times differ
    slightly; stiff components move over that difference)."""
    st = gb.get_state()
    z = st["z"].cpu().numpy()
    s = (t - st["t"]) / st["h"]
    y = np.zeros(z.shape[1])
    for j in range(st["q"], -1, -1):
        y = y * s + z[j]
    return y


def tight_reference(orc, p, t):
    """Oracle run (FP64 LU) with rtol and atol 1e-3 of the problem's, to t
    (cached per problem and time)."""
    key = (p.label, p.ncells, float(p.rtol), float(t))
    if key not in _REF_CACHE:
        ref = orc.Bdf(p, rtol=p.rtol * 1e-3, atol=p.atol * 1e-3)
        assert ref.integrate(t) == 0
        _REF_CACHE[key] = ref.y()
    return _REF_CACHE[key]


def _report(label, yg, yo, p):
    d = wrms_diff(yg, yo, p.rtol, p.atol)
    n = p.uniform_n
    if n:
        pc = cell_wrms(yg, yo, p.rtol, p.atol, n)
        return d, f"wrms diff {d:.3e} (per cell: median {np.median(pc):.3e}, max {pc.max():.3e})"
    return d, f"wrms diff {d:.3e}"


def compare_trajectory(orc, dev, G, p, max_steps=None, okw=None, bar_per_step=END_BAR_PER_STEP,
                       **kw):
    """Lockstep parity of one trajectory (to p.t_end, or over its first
    max_steps accepted steps).  The oracle and the GPU integrator take one
    accepted step at a time; after every step the attempt and
    Newton-iteration counters, the order and the step sizes (the one just
    taken and the next) are compared.

    * While every decision agrees: the states agree within
      END_BAR0 + END_BAR_PER_STEP * k WRMS at a common time after k steps
      (every 32 steps, and at the end; the GPU state is carried to the
      oracle's time along its own Nordsieck history); the largest relative
      step-size difference is printed.
    * At the first step where a decision differs (attempts, iterations,
      order, Newton-matrix setups) or the step sizes have drifted apart
      beyond FLIP_H, the step,
      both sides' decisions and the oracle's threshold quantities (error estimate
      against 1, order-change estimates, the proposed growth factor
      against the 1.5 hysteresis) are printed; the last common state
      before it agreed within the bar above; both runs then continue
      independently to the same end time, where the GPU's error against a
      tight-tolerance oracle run must be within FLIP_ERR_RATIO of the
      oracle's own error (their direct difference is printed), with step
      counts within 15%.

    okw: extra oracle options (e.g. the learned mode's network); kw: GPU
    handle options (linsol and refine_max_it go to both sides); bar_per_step
    replaces END_BAR_PER_STEP (END_BAR_PER_STEP_LAZY for the lazy Newton
    matrix)."""
    lin = kw.pop("linsol", 0)
    rmi = kw.get("refine_max_it", 5)
    ob = orc.Bdf(p, linsol=lin, refine_max_it=rmi, **(okw or {}))
    gb = gpu_bdf(G, p, dev, linsol=lin, **kw)
    k, hdev, flip, snap = 0, 0.0, None, None
    while True:
        rc = ob.step(p.t_end)
        assert rc == 0, rc
        tg = gb.step(p.t_end)
        k += 1
        so, sc, sg = ob.stats(), ob.scalars(), gb.stats()
        dg, do = _decisions(sg, {**so, "q": sc["q"]})
        rel = max(abs(sg["hu"] - sc["hu"]) / abs(sc["hu"]), abs(sg["h"] - sc["h"]) / abs(sc["h"]))
        if dg != do or rel > FLIP_H:
            flip = dict(step=k, t=sc["t"],
                        gpu=dict(att_it_q=dg, t=tg, h=sg["h"], hu=sg["hu"], err=sg["err_last"]),
                        oracle=dict(att_it_q=do, h=sc["h"], hu=sc["hu"], err=sc["err_last"],
                                    err_qm1=sc["err_qm1"], err_qp1=sc["err_qp1"],
                                    eta_proposed=sc["eta_proposed"], q_proposed=sc["q_proposed"]),
                        rel_h=rel)
            break
        hdev = max(hdev, rel)
        if sc["t"] == p.t_end or (max_steps and k >= max_steps):
            break
        if k % 32 == 0:
            yg = gpu_y_at(gb, sc["t"])
            dsnap, _ = _report(p.label, yg, ob.y(), p)
            assert dsnap <= END_BAR0 + bar_per_step * k, (k, sc["t"], dsnap)
            snap = (k, sc["t"], yg, ob.y())
    if flip is None:
        sof, sgf = ob.stats(), gb.stats()
        assert sof["nsteps"] == sgf["nsteps"] and sof["order_hist"] == sgf["order_hist"]
        yg = gb.y().cpu().numpy() if tg == sc["t"] else gpu_y_at(gb, sc["t"])
        d, msg = _report(p.label, yg, ob.y(), p)
        print(f"{p.label}: {k} steps to t = {sc['t']:.6e}, identical decisions; max rel "
              f"step-size difference {hdev:.2e}; state {msg}")
        assert d <= END_BAR0 + bar_per_step * k
        return ob, gb
    print(f"{p.label}: decision flip {flip}; max rel step-size difference before it {hdev:.2e}")
    if snap is not None:
        ks, ts, yg0, yo0 = snap
        dpre, msg = _report(p.label, yg0, yo0, p)
        print(f"  last common state, step {ks}, t = {ts:.6e}: {msg}")
    if max_steps:
        while ob.stats()["nsteps"] < max_steps and ob.scalars()["t"] < p.t_end:
            assert ob.step(p.t_end) == 0
        while ob.scalars()["t"] < tg and ob.scalars()["t"] < p.t_end:
            assert ob.step(p.t_end) == 0
        t_cmp = ob.scalars()["t"]
    else:
        t_cmp = p.t_end
        assert ob.integrate(t_cmp) == 0
    assert gb.integrate(t_cmp) == t_cmp
    so, sg = ob.stats(), gb.stats()
    yg, yo = gb.y().cpu().numpy(), ob.y()
    d, msg = _report(p.label, yg, yo, p)
    yr = tight_reference(orc, p, t_cmp)
    eg, eo = wrms_diff(yg, yr, p.rtol, p.atol), wrms_diff(yo, yr, p.rtol, p.atol)
    print(f"  at t = {t_cmp:.6e}: steps oracle {so['nsteps']} gpu {sg['nsteps']}, gpu vs oracle "
          f"{msg}; error vs tight reference: gpu {eg:.3e}, oracle {eo:.3e}")
    assert eg <= FLIP_ERR_RATIO * eo
    assert abs(so["nsteps"] - sg["nsteps"]) <= max(3, 0.15 * so["nsteps"])
    return ob, gb
