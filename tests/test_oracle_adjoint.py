"""Pins of the oracle's adjoint of the fine step: the linear forms of the
image rule reproduce the stencil values; the momentum adjoint passes the
dot-product test against central differences of the forward predictor; the
gradient of the kinetic energy after several projection steps agrees with
central finite differences of the forward solve to 1e-6."""
import numpy as np
import pytest

from paper_1705_06149_amd import inputs


def _mask():
    n = 10
    solid = np.zeros((n, n, n), np.uint8)
    solid[3:6, 4:6, 2:5] = 1
    solid[7, 2, 6] = 1
    solid[2:4, 7, 7:9] = 1
    return solid


def test_stencil_forms_match_stencil_values(oracle):
    n = 10
    rng = np.random.default_rng(3)
    g = oracle.Grid(n, n, n, solid=_mask(), lid=1 + rng.standard_normal((n, n + 1)))
    st = inputs.random_state(n, n, n, seed=4)
    masks = oracle._open_masks(g)
    checked = 0
    for c in range(3):
        phi = st[c]
        for f in zip(*np.nonzero(masks[c])):
            k, j, i = f
            for d in range(3):
                for m in (-2, -1, 1, 2):
                    a = oracle.stencil_value(g, c, phi, (i, j, k), d, m)
                    b = oracle.stencil_value(g, c, phi, (i, j, k), d, m, as_form=True)
                    assert a == pytest.approx(b, rel=1e-14, abs=1e-14)
                    checked += 1
    assert checked > 20000


@pytest.mark.parametrize("obstacles", [False, True])
def test_momentum_adjoint_dot_product(oracle, obstacles):
    n, dt = 10, 2e-3
    rng = np.random.default_rng(5)
    g = oracle.Grid(n, n, n, re=50.0, solid=_mask() if obstacles else None,
                    lid=1 + 0.2 * rng.standard_normal((n, n + 1)))
    u = inputs.random_state(n, n, n, seed=6, scale=0.5)[:3]
    du = inputs.random_state(n, n, n, seed=7)[:3]
    mu = inputs.random_state(n, n, n, seed=8)[:3]
    masks = oracle._open_masks(g)
    mu = [np.where(m, x, 0.0) for x, m in zip(mu, masks)]
    lam, glid = oracle.momentum_adjoint(g, *u, dt, mu)
    eps = 1e-7
    Fp = oracle.momentum(g, *[a + eps * b for a, b in zip(u, du)], dt)
    Fm = oracle.momentum(g, *[a - eps * b for a, b in zip(u, du)], dt)
    lhs = sum(float(np.sum((p - q) / (2 * eps) * m)) for p, q, m in zip(Fp, Fm, mu))
    rhs = sum(float(np.sum(x[mk] * y[mk])) for x, y, mk in zip(du, lam, masks))
    assert lhs == pytest.approx(rhs, rel=1e-6)
    # lid direction
    dl = rng.standard_normal(g.lid.shape)
    lid0 = g.lid.copy()
    g.lid = lid0 + eps * dl
    Fp = oracle.momentum(g, *u, dt)
    g.lid = lid0 - eps * dl
    Fm = oracle.momentum(g, *u, dt)
    g.lid = lid0
    lhs = sum(float(np.sum((p - q) / (2 * eps) * m)) for p, q, m in zip(Fp, Fm, mu))
    assert lhs == pytest.approx(float(np.sum(dl * glid)), rel=1e-6)


def test_kinetic_energy_gradient_matches_finite_differences(oracle):
    n, steps, dt = 10, 6, 1e-3
    g = oracle.Grid(n, n, n, re=400.0)
    u0 = inputs.div_free_perturbation(n, n, n, seed=5, sigma=1e-2)
    st0 = (u0[0], u0[1], u0[2], np.zeros((n, n, n)))
    J, grad, glid = oracle.adjoint_gradient(g, st0, steps, dt, ckpt_every=4)
    rng = np.random.default_rng(7)
    d = inputs.div_free_perturbation(n, n, n, seed=9, sigma=1e-2)
    masks = oracle._open_masks(g)
    pred = sum(float(np.sum(a[m] * b[m])) for a, b, m in zip(grad, d, masks))

    def Jof(state, lid=None):
        gg = oracle.Grid(n, n, n, re=400.0, lid=lid)
        y = state
        for _ in range(steps):
            y, _, _, _ = oracle.fine_steps(gg, y, 1, dt, rtol=1e-13)
        return oracle.kinetic_energy(gg, y)

    # inside the plateau between SMART branch flips (larger steps) and
    # round-off (smaller steps): 1e-5 and 1e-6 agree to ~2e-9 here
    eps = 1e-5
    sp = tuple(a + eps * b for a, b in zip(u0, d)) + (np.zeros((n, n, n)),)
    sm = tuple(a - eps * b for a, b in zip(u0, d)) + (np.zeros((n, n, n)),)
    fd = (Jof(sp) - Jof(sm)) / (2 * eps)
    assert fd == pytest.approx(pred, rel=1e-6)
    # lid profile direction: sum of sine modes
    B = inputs.lid_profile_basis(n, n, nmodes=3)
    dl = B[0, 0] + 0.5 * B[1, 2] - 0.3 * B[2, 1]
    fd = (Jof(st0, np.ones((n, n + 1)) + eps * dl) - Jof(st0, np.ones((n, n + 1)) - eps * dl)) / (2 * eps)
    assert fd == pytest.approx(float(np.sum(glid * dl)), rel=1e-6)
    # checkpointing does not change the result
    J2, grad2, glid2 = oracle.adjoint_gradient(g, st0, steps, dt, ckpt_every=None)
    assert J2 == J and all(np.array_equal(a, b) for a, b in zip(grad, grad2)) and np.array_equal(glid, glid2)
