"""Pins of the oracle's multi-time-step loop with beam evolution: test
electrons in a pure ion column oscillate at the betatron wavenumber
k_beta = 1/sqrt(2 gamma) (normalised units: the ion column of density n0 = 1
focuses with Ex - By = x/2), and a step keeps each beam particle in the slice
it had at the start of the box."""
import numpy as np

import workloads as W
from oracle import qsp_oracle as O


def dead_plasma(cfg):
    st = O.initial_state(cfg)
    st.plasma.w[:] = 0.0
    return st


def run_column(nsteps, **kw):
    cfg, beam = W.ion_column(**kw)
    xs, ys = [beam.x.astype(np.float64).copy()], [beam.y.astype(np.float64).copy()]

    def after(step, recs):
        xs.append(beam.x.astype(np.float64).copy())
        ys.append(beam.y.astype(np.float64).copy())
    O.run_steps(cfg, beam, nsteps, state_fn=lambda: dead_plasma(cfg), after_step=after)
    return cfg, beam, np.array(xs), np.array(ys)


def test_ion_column_field_is_half_the_offset():
    cfg, _ = W.ion_column()
    recs, _ = O.run_box(cfg, None, state=dead_plasma(cfg), k_end=1)
    x, y = O.node_coords(cfg)
    near = (np.abs(x) < 0.6)
    row = cfg.ny // 2
    slope = np.polyfit(x[near], recs[0]["exmby"][row, near], 1)[0]
    # the square box with psi = 0 on its walls adds an O((r/L)^2) harmonic correction
    assert abs(slope - 0.5) < 5e-3, slope
    assert np.abs(recs[0]["ez"]).max() < 1e-12


def test_betatron_oscillation_in_ion_column():
    gamma, dt, x0, nsteps = 2000.0, 6.0, 0.2, 200
    cfg, beam, xs, ys = run_column(nsteps, gamma=gamma, dt=dt, x0=x0)
    t = dt * np.arange(nsteps + 1)
    kb = 1.0 / np.sqrt(2.0 * gamma)
    # particle 0 starts at (x0, 0): x = x0 cos(k_beta t), y = 0
    assert np.max(np.abs(xs[:, 0] - x0 * np.cos(kb * t))) < 0.03 * x0
    assert np.max(np.abs(ys[:, 0])) < 1e-6
    # frequency from a least-squares fit of cos/sin over the whole record
    for p in range(cfg.nzeta):
        for series, start in ((xs[:, p], xs[0, p]), (ys[:, p], ys[0, p])):
            if abs(start) < 1e-6:
                continue
            ks = np.linspace(0.97 * kb, 1.03 * kb, 601)
            resid = [np.linalg.lstsq(np.stack([np.cos(k * t), np.sin(k * t)], 1), series,
                                     rcond=None)[1][0] for k in ks]
            k_fit = ks[int(np.argmin(resid))]
            assert abs(k_fit / kb - 1.0) < 3e-3, (p, k_fit / kb)


def test_betatron_period_shrinks_with_sqrt_gamma():
    # k_beta scales as gamma^(-1/2): quarter period at gamma and 4 gamma
    quarter = []
    for gamma in (500.0, 2000.0):
        kb = 1.0 / np.sqrt(2.0 * gamma)
        n = int(np.ceil(0.5 * np.pi / kb / 6.0)) + 2
        _, _, xs, _ = run_column(n, gamma=gamma)
        t = 6.0 * np.arange(n + 1)
        s = xs[:, 0]
        i = int(np.nonzero(s < 0)[0][0])            # first zero crossing
        quarter.append(t[i - 1] + s[i - 1] / (s[i - 1] - s[i]) * 6.0)
    assert abs(quarter[1] / quarter[0] - 2.0) < 0.02, quarter


def test_a_step_keeps_the_slice_assignment_of_its_start():
    # identical test electrons in slices 1 and 3; the one in slice 1 sits just
    # ahead of the slice boundary and drifts across it during the step: it is
    # still deposited and pushed once, in its starting slice, so both move alike
    cfg, beam = W.ion_column(nzeta=4)
    beam.x[:] = np.float32(0.1)
    beam.y[:] = np.float32(0.0)
    beam.uz[:] = np.float32(10.0)                     # slow: drifts back by dt (u_z/gamma - 1)
    zeta0 = np.asarray(cfg.zeta(), dtype=np.float32)
    zeta0[1] = np.float32(cfg.zeta_hi - 1.5 * cfg.dzeta + 2e-6)
    beam.zeta[:] = zeta0
    before = O.beam_slice_index(cfg, beam.zeta).copy()
    O.run_steps(cfg, beam, 1, state_fn=lambda: dead_plasma(cfg))
    after = O.beam_slice_index(cfg, beam.zeta)
    assert before[1] == 1 and after[1] == 2           # crossed during the step
    d = beam.zeta.astype(np.float64) - zeta0.astype(np.float64)
    assert abs(d[1] - d[3]) < 1e-6, d                 # one push each
    assert abs(beam.x[1] - beam.x[3]) < 1e-7 and abs(beam.uz[1] - beam.uz[3]) < 1e-5
