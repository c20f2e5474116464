"""Plain FP64 reference of the learned warm start (bipartite message passing
network over the constraint graph of an LP).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: the HIP network
kernels are checked against these functions; the product path never imports
them.  Written with numpy, one LP at a time, no fusion and no blocking.

Model (hidden width H = 64, L = 3 rounds), for an LP min c'x s.t. rows of
A x (=, >=, <=) b, l <= x <= u, with constraint nodes i and variable nodes j
joined by the nonzeros a_ij:

  scales     s_c = max|c|, s_b = max|b|, s_a = max|a_ij| (1 where the max is 0)
  features   f_v[j] = (c_j/s_c, l_j/s_b or 0, u_j/s_b or 0, [l_j finite], [u_j finite])
             f_c[i] = (b_i/s_b, [EQ], [GE], [LE])
  edges      w_ij = a_ij / s_a; d_i, d_j = nonzeros of row i / column j (>= 1)
  embed      h_v = relu(f_v W_v0 + b_v0),   h_c = relu(f_c W_c0 + b_c0)
  round r    m_c = diag(1/d_i) W h_v;    h_c = relu([h_c | m_c] Phi_r + phi_r)
             m_v = diag(1/d_j) W' h_c;   h_v = relu([h_v | m_v] Psi_r + psi_r)
  heads      xh = h_v w_x + b_x,  yh = h_c w_y + b_y,
             oh = [mean_j h_v | mean_i h_c] w_o + b_o
  outputs    x0 = xh s_b/s_a,  y0 = yh s_c/s_a,  omega0 = exp(oh)

Loss of one LP against a solution (x*, y*, omega*), with term weights
(w_x, w_y, w_o), 1 by default:
  w_x mean_j (xh_j - x*_j s_a/s_b)^2 + w_y mean_i (yh_i - y*_i s_a/s_c)^2 + w_o (oh - log omega*)^2,
averaged over the LPs of a mini-batch; Adam (Kingma & Ba) on FP32 master
weights.  With ``bf16=True`` the operands of the eight 128 x 64 products (forward
and both backward products) are rounded to bfloat16 (round to nearest even)
before the FP64 product, as the MFMA kernels take them; everything else stays
FP64.
"""
from __future__ import annotations

import numpy as np

H = 64
ROUNDS = 3
DV, DC = 5, 4

# parameter names and shapes, in the order of the flat parameter vector
PARAMS = ([("W_v0", (DV, H)), ("b_v0", (H,)), ("W_c0", (DC, H)), ("b_c0", (H,))]
          + [p for r in range(ROUNDS) for p in ((f"Phi{r}", (2 * H, H)), (f"phi{r}", (H,)),
                                                 (f"Psi{r}", (2 * H, H)), (f"psi{r}", (H,)))]
          + [("w_x", (H,)), ("b_x", (1,)), ("w_y", (H,)), ("b_y", (1,)), ("w_o", (2 * H,)), ("b_o", (1,))])
N_PARAMS = sum(int(np.prod(s)) for _, s in PARAMS)


def unflatten(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in PARAMS:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in PARAMS])


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits), ties to even."""
    a = np.asarray(a, np.float64)
    m, e = np.frexp(a)                 # a = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round: half to even


def graph(prob) -> dict:
    """Features, edge weights and degrees of one LP (see the module doc)."""
    m, n = int(prob.m), int(prob.n)
    rp = np.asarray(prob.row_ptr, np.int64)
    ci = np.asarray(prob.col_idx, np.int64)
    a = np.asarray(prob.val, np.float64)
    c, b = np.asarray(prob.c, np.float64), np.asarray(prob.b, np.float64)
    l, u = np.asarray(prob.l, np.float64), np.asarray(prob.u, np.float64)
    s_c = float(np.max(np.abs(c))) if n else 0.0
    s_b = float(np.max(np.abs(b))) if m else 0.0
    s_a = float(np.max(np.abs(a))) if len(a) else 0.0
    s_c, s_b, s_a = (s if s > 0 else 1.0 for s in (s_c, s_b, s_a))
    lf, uf = np.isfinite(l), np.isfinite(u)
    f_v = np.stack([c / s_c, np.where(lf, l, 0.0) / s_b, np.where(uf, u, 0.0) / s_b,
                    lf.astype(float), uf.astype(float)], axis=1)
    rt = np.asarray(prob.row_type)
    f_c = np.stack([b / s_b, (rt == 0).astype(float), (rt == 1).astype(float), (rt == 2).astype(float)], axis=1)
    rows = np.repeat(np.arange(m), np.diff(rp))
    W = np.zeros((m, n))
    W[rows, ci] = a / s_a
    d_c = np.maximum(1, np.diff(rp)).astype(float)
    d_v = np.maximum(1, np.bincount(ci, minlength=n)).astype(float)
    return dict(m=m, n=n, f_v=f_v, f_c=f_c.reshape(m, DC), W=W, d_c=d_c, d_v=d_v, s_c=s_c, s_b=s_b, s_a=s_a)


def _mm(x, w, q):
    return (bf16(x) @ bf16(w)) if q else (x @ w)


def forward(p: dict, g: dict, bf16_ops: bool = False):
    """(xh[n], yh[m], oh, cache) for one LP."""
    relu = lambda z: np.maximum(z, 0.0)
    zv0 = g["f_v"] @ p["W_v0"] + p["b_v0"]
    zc0 = g["f_c"] @ p["W_c0"] + p["b_c0"]
    hv, hc = relu(zv0), relu(zc0)
    cache = dict(zv0=zv0, zc0=zc0, rounds=[])
    for r in range(ROUNDS):
        mc = (g["W"] @ hv) / g["d_c"][:, None]
        xc = np.concatenate([hc, mc], axis=1)
        zc = _mm(xc, p[f"Phi{r}"], bf16_ops) + p[f"phi{r}"]
        hc_new = relu(zc)
        mv = (g["W"].T @ hc_new) / g["d_v"][:, None]
        xv = np.concatenate([hv, mv], axis=1)
        zv = _mm(xv, p[f"Psi{r}"], bf16_ops) + p[f"psi{r}"]
        hv_new = relu(zv)
        cache["rounds"].append(dict(xc=xc, zc=zc, xv=xv, zv=zv))
        hv, hc = hv_new, hc_new
    xh = hv @ p["w_x"] + p["b_x"][0]
    yh = hc @ p["w_y"] + p["b_y"][0]
    pool = np.concatenate([hv.mean(axis=0), hc.mean(axis=0) if g["m"] else np.zeros(H)])
    oh = float(pool @ p["w_o"] + p["b_o"][0])
    cache.update(hv=hv, hc=hc, pool=pool)
    return xh, yh, oh, cache


def targets(g: dict, x_star, y_star, omega_star):
    """Targets in the network's units."""
    return (np.asarray(x_star, float) * g["s_a"] / g["s_b"], np.asarray(y_star, float) * g["s_a"] / g["s_c"],
            float(np.log(omega_star)))


def predictions(g: dict, xh, yh, oh):
    """(x0, y0, omega0) in the LP's units."""
    return xh * g["s_b"] / g["s_a"], yh * g["s_c"] / g["s_a"], float(np.exp(oh))


def loss_one(g, xh, yh, oh, t, wts=(1.0, 1.0, 1.0)):
    """w_x mean_j (xh - xt)^2 + w_y mean_i (yh - yt)^2 + w_o (oh - ot)^2."""
    xt, yt, ot = t
    wx, wy, wo = wts
    L = (wx * float(np.mean((xh - xt) ** 2)) + (wy * float(np.mean((yh - yt) ** 2)) if g["m"] else 0.0)
         + wo * (oh - ot) ** 2)
    return L


def backward(p: dict, g: dict, cache: dict, xh, yh, oh, t, scale: float = 1.0, bf16_ops: bool = False,
             wts=(1.0, 1.0, 1.0)) -> dict:
    """Gradient of scale * loss_one with respect to every parameter."""
    xt, yt, ot = t
    wx, wy, wo = wts
    n, m = g["n"], g["m"]
    grads = {name: np.zeros(shape) for name, shape in PARAMS}
    dxh = scale * wx * 2.0 * (xh - xt) / n
    dyh = scale * wy * 2.0 * (yh - yt) / m if m else np.zeros(0)
    doh = scale * wo * 2.0 * (oh - ot)
    hv, hc = cache["hv"], cache["hc"]
    grads["w_x"] = hv.T @ dxh
    grads["b_x"] = np.array([dxh.sum()])
    grads["w_y"] = hc.T @ dyh if m else np.zeros(H)
    grads["b_y"] = np.array([dyh.sum()])
    grads["w_o"] = doh * cache["pool"]
    grads["b_o"] = np.array([doh])
    dhv = np.outer(dxh, p["w_x"]) + doh * p["w_o"][:H] / n
    dhc = np.outer(dyh, p["w_y"]) + (doh * p["w_o"][H:] / m if m else 0.0)
    for r in reversed(range(ROUNDS)):
        c = cache["rounds"][r]
        # variable update: hv = relu([hv_in | mv] Psi + psi), mv = W' hc / d_v
        dzv = dhv * (c["zv"] > 0)
        grads[f"Psi{r}"] = _mm(c["xv"].T, dzv, bf16_ops)
        grads[f"psi{r}"] = dzv.sum(axis=0)
        dxv = _mm(dzv, p[f"Psi{r}"].T, bf16_ops)
        dhv_in, dmv = dxv[:, :H], dxv[:, H:]
        dhc = dhc + g["W"] @ (dmv / g["d_v"][:, None])
        # constraint update: hc = relu([hc_in | mc] Phi + phi), mc = W hv_in / d_c
        dzc = dhc * (c["zc"] > 0)
        grads[f"Phi{r}"] = _mm(c["xc"].T, dzc, bf16_ops)
        grads[f"phi{r}"] = dzc.sum(axis=0)
        dxc = _mm(dzc, p[f"Phi{r}"].T, bf16_ops)
        dhc_in, dmc = dxc[:, :H], dxc[:, H:]
        dhv = dhv_in + g["W"].T @ (dmc / g["d_c"][:, None])
        dhc = dhc_in
    dzv0 = dhv * (cache["zv0"] > 0)
    dzc0 = dhc * (cache["zc0"] > 0)
    grads["W_v0"] = g["f_v"].T @ dzv0
    grads["b_v0"] = dzv0.sum(axis=0)
    grads["W_c0"] = g["f_c"].T @ dzc0
    grads["b_c0"] = dzc0.sum(axis=0)
    return grads


def batch_loss_and_grad(theta: np.ndarray, graphs, tgts, bf16_ops: bool = False, wts=(1.0, 1.0, 1.0)):
    """Mean loss over the LPs and its gradient (flat vectors)."""
    p = unflatten(theta)
    K = len(graphs)
    total = 0.0
    acc = np.zeros(N_PARAMS)
    for g, t in zip(graphs, tgts):
        xh, yh, oh, cache = forward(p, g, bf16_ops)
        total += loss_one(g, xh, yh, oh, t, wts) / K
        acc += flatten(backward(p, g, cache, xh, yh, oh, t, 1.0 / K, bf16_ops, wts))
    return total, acc


def adam(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
