"""Pins of the network reference in oracle/gnn.py (CPU).

Each check ties the reference to something other than itself: central finite
differences of the loss for the hand-written backward; closed forms of the
forward with chosen weights; equivariance under renumbering; the bfloat16
rounding against a float32 bit-level rounding; Adam's first step."""
import numpy as np
import pytest

import lpgen
from oracle import gnn


def _lp():
    return lpgen.mixed_lp(4, m=7, n=9, density=0.35)


def _theta(seed=1):
    th = lpgen.gnn_init(seed, gnn.PARAMS)
    # nonzero biases so every term of the backward is exercised
    rng = np.random.default_rng(seed)
    p = gnn.unflatten(th)
    for name, shape in gnn.PARAMS:
        if name.startswith(("b_", "phi", "psi")):
            p[name] = 0.1 * rng.standard_normal(shape)
    return gnn.flatten(p)


def _targets(g, rng):
    return (rng.standard_normal(g["n"]), rng.standard_normal(g["m"]), float(rng.standard_normal()))


def test_parameter_count():
    assert gnn.N_PARAMS == 5 * 64 + 64 + 4 * 64 + 64 + 3 * 2 * (128 * 64 + 64) + 64 + 1 + 64 + 1 + 128 + 1


@pytest.mark.parametrize("which", ["mixed", "box", "transport"])
def test_gradient_matches_finite_differences(which):
    rng = np.random.default_rng(7)
    if which == "mixed":
        probs = [_lp(), lpgen.mixed_lp(5, m=5, n=6, density=0.5)]
    elif which == "box":   # no rows: the y head and the constraint pool drop out
        z = np.zeros(0)
        probs = [lpgen.Problem(0, 4, np.zeros(1, np.int32), np.zeros(0, np.int32), z,
                               np.array([1.0, -2.0, 0.5, 3.0]), z, np.zeros(4), np.full(4, 2.0),
                               np.zeros(0, np.int8))]
    else:
        probs = [lpgen.transport_family_lp(0, 0, 3, 4)]
    graphs = [gnn.graph(p) for p in probs]
    tgts = [_targets(g, rng) for g in graphs]
    theta = _theta()
    wts = (2.0, 0.5, 0.25)
    L, grad = gnn.batch_loss_and_grad(theta, graphs, tgts, wts=wts)
    # every embedding, bias and head coordinate plus a sample of the round
    # matrices; a coordinate whose step crosses a ReLU kink (the one-sided
    # differences disagree) is not differentiable there and is left out
    names = np.concatenate([[nm] * int(np.prod(sh)) for nm, sh in gnn.PARAMS])
    small = np.flatnonzero([not (nm.startswith("Phi") or nm.startswith("Psi")) for nm in names])
    idx = np.union1d(small, rng.choice(gnn.N_PARAMS, 400, replace=False))
    f = lambda t: gnn.batch_loss_and_grad(t, graphs, tgts, wts=wts)[0]
    h = 1e-6
    kinks, errs = 0, []
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        lp, lm = f(tp), f(tm)
        fwd, bwd = (lp - L) / h, (L - lm) / h
        if abs(fwd - bwd) > 1e-4 * (1 + abs(fwd)):
            kinks += 1
            continue
        fd = (lp - lm) / (2 * h)
        errs.append(abs(fd - grad[i]) / (1 + abs(fd)))
    assert kinks <= len(idx) // 100, kinks
    assert max(errs) <= 1e-6, max(errs)
    assert L > 0


def test_loss_weights_scale_the_terms():
    g = gnn.graph(_lp())
    rng = np.random.default_rng(1)
    xh, yh, oh = rng.standard_normal(g["n"]), rng.standard_normal(g["m"]), 0.3
    t = _targets(g, rng)
    ex = np.mean((xh - t[0]) ** 2); ey = np.mean((yh - t[1]) ** 2); eo = (oh - t[2]) ** 2
    assert gnn.loss_one(g, xh, yh, oh, t) == pytest.approx(ex + ey + eo, rel=1e-14)
    assert gnn.loss_one(g, xh, yh, oh, t, (3.0, 0.0, 0.5)) == pytest.approx(3 * ex + 0.5 * eo, rel=1e-14)


def test_forward_closed_form():
    """Embeddings pass (c/s_c) and (b/s_b) through channel 0; one round with
    Phi taking the message and Psi the state; the heads read channel 0."""
    A = np.array([[2.0, 0.0, -1.0], [0.0, 4.0, 1.0]])
    c = np.array([3.0, -1.0, 1.5])
    b = np.array([1.0, -2.0])
    p = lpgen.from_dense(A, c, b, np.zeros(3), np.full(3, np.inf), [0, 1])
    g = gnn.graph(p)
    P = {name: np.zeros(shape) for name, shape in gnn.PARAMS}
    P["W_v0"][0, 0] = 1.0      # h_v[:, 0] = relu(c / 3)
    P["W_c0"][0, 0] = 1.0      # h_c[:, 0] = relu(b / 2)
    for r in range(gnn.ROUNDS):
        P[f"Phi{r}"][64, 0] = 1.0   # h_c[:, 0] = relu(m_c[:, 0])
        P[f"Psi{r}"][0, 0] = 1.0    # h_v[:, 0] = relu(h_v[:, 0])
    P["w_x"][0] = 1.0
    P["w_y"][0] = 1.0
    P["w_o"][0] = 2.0
    P["w_o"][64] = 1.0
    P["b_o"][0] = 0.5
    xh, yh, oh, _ = gnn.forward(P, g)
    hv = np.maximum(c / 3.0, 0.0)                        # (1, 0, 0.5), unchanged by the rounds
    W = A / 4.0                                          # s_a = 4
    mc = (W @ hv) / np.array([2.0, 2.0])                 # two nonzeros per row
    hc = np.maximum(mc, 0.0)
    np.testing.assert_allclose(xh, hv, rtol=0, atol=1e-15)
    np.testing.assert_allclose(yh, hc, rtol=0, atol=1e-15)
    assert oh == pytest.approx(2.0 * hv.mean() + hc.mean() + 0.5, abs=1e-15)
    x0, y0, w0 = gnn.predictions(g, xh, yh, oh)
    np.testing.assert_allclose(x0, xh * 2.0 / 4.0)      # s_b / s_a
    np.testing.assert_allclose(y0, yh * 3.0 / 4.0)      # s_c / s_a
    assert w0 == pytest.approx(np.exp(oh))


def test_equivariance_under_renumbering():
    p = _lp()
    P = gnn.unflatten(_theta(3))
    xh, yh, oh, _ = gnn.forward(P, gnn.graph(p))
    rng = np.random.default_rng(0)
    rp, cp = rng.permutation(p.m), rng.permutation(p.n)
    xq, yq, oq, _ = gnn.forward(P, gnn.graph(lpgen.permute(p, rp, cp)))
    np.testing.assert_allclose(xq, xh[cp], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(yq, yh[rp], rtol=1e-12, atol=1e-14)
    assert oq == pytest.approx(oh, rel=1e-12)


def _bf16_bits(a):
    """bfloat16 rounding of float32 values by the bit pattern (round to
    nearest even on the 16 dropped bits)."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def test_bf16_rounding():
    assert gnn.bf16(np.array([1.0]))[0] == 1.0
    assert gnn.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0            # tie -> even
    assert gnn.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6   # tie -> even (up)
    assert gnn.bf16(np.array([1.0 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    assert gnn.bf16(np.array([-0.0]))[0] == 0.0
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    np.testing.assert_array_equal(gnn.bf16(a.astype(np.float64)), _bf16_bits(a))


def test_bf16_products_close_to_fp64():
    """Rounding the product operands to bfloat16 moves the outputs by about
    the bfloat16 unit (2^-8) relative, not more."""
    probs = [lpgen.transport_family_lp(0, k, 10, 10) for k in range(2)]
    P = gnn.unflatten(_theta(5))
    for p in probs:
        g = gnn.graph(p)
        a = gnn.forward(P, g)
        b = gnn.forward(P, g, bf16_ops=True)
        for u, v in ((a[0], b[0]), (a[1], b[1])):
            assert np.linalg.norm(u - v) <= 2e-2 * np.linalg.norm(u)
        assert abs(a[2] - b[2]) <= 2e-2 * (1 + abs(a[2]))


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(0)
    th = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = gnn.adam(th, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    # g / (|g| + eps) differs from sign(g) by eps / |g|
    assert np.all(np.abs(new - (th - 1e-3 * np.sign(g))) <= 1e-3 * 1e-8 / np.abs(g) + 1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    """A few Adam steps on a tiny family lower the loss (the reference can learn)."""
    probs = [lpgen.transport_family_lp(1, k, 4, 5) for k in range(4)]
    graphs = [gnn.graph(p) for p in probs]
    rng = np.random.default_rng(2)
    tgts = [(np.abs(rng.standard_normal(g["n"])), rng.standard_normal(g["m"]), 0.3) for g in graphs]
    th = _theta(6)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    L0 = gnn.batch_loss_and_grad(th, graphs, tgts)[0]
    for step in range(1, 61):
        L, gr = gnn.batch_loss_and_grad(th, graphs, tgts)
        th, m, v = gnn.adam(th, gr, m, v, step, lr=3e-3)
    assert gnn.batch_loss_and_grad(th, graphs, tgts)[0] < 0.7 * L0
