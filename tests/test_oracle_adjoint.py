"""Pins of the gradient oracle (oracle/adjoint.py).

* Its kernel polynomials equal the C oracle's W, F = dW/dr and dW/dh for the
  M4, M6 and Wendland C6 kernels of Sect. 2.3, and its written-out df/dq
  equals autograd of f.
* Its forward evaluation and K-step leapfrog rollout reproduce the C
  oracle's values (Sect. 2.2-2.6, Sect. 2.4).
* Its gradients match central finite differences of the C oracle, which
  re-solves every h and re-finds every neighbour set: the vector-Jacobian
  product of one evaluation along random directions, and the gradient of
  sum m|a|^2 + kinetic energy after K steps, per component on sampled
  particles and along a random direction.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint as adj
from paper_1909_07439_amd import inputs

KINDS = [oracle.M4, oracle.M6, oracle.WENDLAND_C6]
FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u")


@pytest.mark.parametrize("kind", KINDS)
def test_kernel_polynomials_match_c_oracle(kind):
    S = oracle.kernel_support(kind)
    r = np.linspace(0.0, S + 0.5, 4001)[1:]
    h = 1.0 + 0.3 * np.sin(7 * r)
    w, F, dh = oracle.kernel(kind, r, h)
    rt, ht = torch.from_numpy(r), torch.from_numpy(h)
    for got, want in ((adj.kernel_w(kind, rt, ht), w), (adj.kernel_F(kind, rt, ht), F),
                      (adj.kernel_dwdh(kind, rt, ht), dh)):
        scale = np.abs(want).max()
        np.testing.assert_allclose(got.numpy(), want, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("kind", KINDS)
def test_written_out_derivative_is_autograd_of_f(kind):
    q = torch.linspace(0.0, oracle.kernel_support(kind) + 0.5, 3001, dtype=torch.float64)
    q.requires_grad_(True)
    (g,) = torch.autograd.grad(adj.kernel_f(kind, q).sum(), q)
    want = adj.kernel_df(kind, q).detach()
    assert torch.max(torch.abs(g - want)) <= 1e-12 * torch.max(torch.abs(want))


def small_state(n_side=8, kind=oracle.M4, seed_variant=0, terms="all"):
    """Jittered lattice with velocities.  u takes two levels (1 and 1.5) at
    random: the conductivity's signal speed sqrt|P_i - P_j| has no derivative
    where P_i = P_j, and with two levels every pair with u_i != u_j (the only
    pairs whose conductivity term depends on that speed to first order) has
    |P_i - P_j| far from zero, so finite differences resolve the gradient.
    ``terms`` switches viscosity and conductivity on or off."""
    c = inputs.with_kernel(inputs.lattice(n_side, jitter=0.3, velocities=True,
                                          seed_variant=seed_variant), kind)
    rng = np.random.default_rng(100 + seed_variant)
    c["u"] = np.where(rng.random(c["n"]) < 0.5, 1.0, 1.5)
    av = terms in ("av", "all")
    c["alpha_av"], c["beta_av"] = (1.0, 2.0) if av else (0.0, 0.0)
    c["alpha_u"] = 1.0 if terms in ("cond", "all") else 0.0
    return c


@pytest.mark.parametrize("kind", KINDS)
def test_forward_evaluation_matches_c_oracle(kind):
    c = small_state(kind=kind)
    p = oracle.make_params(c)
    o = oracle.evaluate(c, p)
    st = {k: torch.from_numpy(np.asarray(c[k], dtype=np.float64)) for k in FIELDS}
    st["h_start"] = c["h"]
    e = adj.evaluate(c, p, st)
    for k in ("h", "rho", "omega"):
        np.testing.assert_allclose(e[k].numpy(), o[k], rtol=1e-13)
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(e[k].numpy() - o[k]) / o["anorm"]) < 1e-12
    assert np.max(np.abs(e["dudt"].numpy() - o["dudt"]) / o["unorm"]) < 1e-12


def c_rollout(c, dt, K, p):
    """The C oracle: initial evaluation and K steps of fixed dt."""
    s = oracle.evaluate(c, p)
    for _ in range(K):
        s = oracle.step(s, dt, p)
    return s


def c_loss(c, dt, K, p):
    s = c_rollout(c, dt, K, p)
    m = c["m"]
    return float(np.sum(m * (s["ax"] ** 2 + s["ay"] ** 2 + s["az"] ** 2)) +
                 np.sum(m * 0.5 * (s["vx"] ** 2 + s["vy"] ** 2 + s["vz"] ** 2)))


def fixed_dt(c, p):
    return 0.5 * oracle.evaluate(c, p)["dt_next"]


def test_rollout_forward_matches_c_oracle():
    c = small_state()
    p = oracle.make_params(c)
    dt = fixed_dt(c, p)
    s = c_rollout(c, dt, 3, p)
    _, out = adj.rollout(c, dt, 3)
    for k in ("x", "y", "z", "vx", "vy", "vz", "u"):
        np.testing.assert_allclose(out[k].detach().numpy(), s[k], rtol=1e-12,
                                   atol=1e-12 * np.abs(s[k]).max())
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(out[k].detach().numpy() - s[k]) / s["anorm"]) < 1e-10


def perturbed(c, delta, eps):
    d = dict(c)
    for k in FIELDS:
        d[k] = c[k] + eps * delta[k]
        if k in ("x", "y", "z"):
            d[k] = np.mod(d[k], 1.0)
    return d


# tolerance on |FD - AD| / sum_k |g_k . delta_k| per set of active terms;
# the conductivity's sqrt|P_i - P_j| leaves kinks that eps = 1e-6 still meets
VJP_TOL = {"pressure": 1e-8, "av": 1e-7, "cond": 1e-5, "all": 1e-5}


@pytest.mark.parametrize("terms", ["pressure", "av", "cond", "all"])
@pytest.mark.parametrize("kind", KINDS)
def test_evaluation_vjp_matches_finite_differences(kind, terms):
    c = small_state(kind=kind, seed_variant=3, terms=terms)
    p = oracle.make_params(c)
    rng = np.random.default_rng(11)
    n = c["n"]
    cot = {k: rng.normal(size=n) for k in ("ax", "ay", "az", "dudt")}
    g, _ = adj.eval_vjp(c, cot)

    def L(cc):
        o = oracle.evaluate(cc, p)
        return sum(float(np.dot(cot[k], o[k])) for k in cot)

    for trial in range(2):
        delta = {k: rng.normal(size=n) for k in FIELDS}
        for k in ("x", "y", "z"):
            delta[k] *= 0.1 * c["dx"]
        eps = 1e-6
        fd = (L(perturbed(c, delta, eps)) - L(perturbed(c, delta, -eps))) / (2 * eps)
        ad = sum(float(np.dot(g[k], delta[k])) for k in FIELDS)
        mag = sum(float(np.abs(g[k] * delta[k]).sum()) for k in FIELDS)
        assert abs(fd - ad) <= VJP_TOL[terms] * mag, (trial, fd, ad, mag)


# the same tolerance per active terms, for the rollout; after the first step
# u no longer takes two levels and the conductivity's kinks come nearer
ROLL_TOL = {"av": 1e-7, "all": 1e-5}


@pytest.mark.parametrize("kind,terms", [(oracle.M4, "av"), (oracle.WENDLAND_C6, "av"),
                                        (oracle.M6, "av"), (oracle.M4, "all")])
def test_rollout_gradient_matches_finite_differences(kind, terms):
    c = small_state(kind=kind, seed_variant=5, terms=terms)
    p = oracle.make_params(c)
    dt = fixed_dt(c, p)
    K = 3
    g, loss = adj.rollout_grad(c, dt, K)
    assert abs(loss - c_loss(c, dt, K, p)) <= 1e-12 * loss
    rng = np.random.default_rng(12)
    eps = 1e-6
    # per component, on sampled particles (the loss is a global sum)
    scale = {k: np.abs(g[k]).max() for k in FIELDS}
    for i in rng.choice(c["n"], 4, replace=False):
        for k in FIELDS:
            delta = {q: np.zeros(c["n"]) for q in FIELDS}
            delta[k][i] = 1.0
            fd = (c_loss(perturbed(c, delta, eps), dt, K, p) -
                  c_loss(perturbed(c, delta, -eps), dt, K, p)) / (2 * eps)
            assert abs(fd - g[k][i]) <= 100 * ROLL_TOL[terms] * scale[k], (i, k, fd, g[k][i])
    # along a random direction
    delta = {k: rng.normal(size=c["n"]) for k in FIELDS}
    for k in ("x", "y", "z"):
        delta[k] *= 0.1 * c["dx"]
    fd = (c_loss(perturbed(c, delta, eps), dt, K, p) -
          c_loss(perturbed(c, delta, -eps), dt, K, p)) / (2 * eps)
    ad = sum(float(np.dot(g[k], delta[k])) for k in FIELDS)
    mag = sum(float(np.abs(g[k] * delta[k]).sum()) for k in FIELDS)
    assert abs(fd - ad) <= ROLL_TOL[terms] * mag, (fd, ad, mag)
