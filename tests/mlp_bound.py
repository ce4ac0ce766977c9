"""A priori bound on how far the picker network's fp32 kernels may lie from the
float64 reference (test infrastructure; used to set the tolerances of the MLP
parity tests).

Forward error analysis in the standard model fl(a op b) = (a op b)(1 + d),
|d| <= u (Higham, Accuracy and Stability of Numerical Algorithms, 2nd ed.,
sections 2.2 and 3.1-3.4).  Expand a value built from + and x (and division by
an exact operand) into monomials of the inputs: each monomial carries a product
of at most k factors (1 + d_i), k the number of roundings on its way, and
|prod (1 + d_i) - 1| <= gamma_k = k u / (1 - k u) (Lemma 3.1).  Hence

    |computed - exact| <= gamma_k * (the same expression evaluated on the
                                     absolute values of its inputs, every
                                     subtraction taken as an addition),

where k, the rounding depth, obeys depth(a + b) = max(depth a, depth b) + 1
and depth(a * b) = depth a + depth b + 1.  A fused multiply-add rounds once
where this count takes two, and any summation order of n terms gives each term
at most n roundings, so the counts below bound the kernels whatever order and
contraction the compiler picks.  fp32 division in these kernels is the
correctly rounded one (one rounding).

Depths, one row of the network y = W3 . relu(W2 relu(W1 xs + b1) + b2) + b3:
  xs = (x - mean) / std                     2
  a1 = b1 + sum of 66 products W1 xs        2 + 1 + 66 = 69
  a2 = b2 + sum of 64 products W2 h1        69 + 1 + 64 = 134
  y  = b3 + W3 . h2 (64 products, a 6-level
       tree, then b3)                        134 + 1 + 6 + 1 = 142
The loss derivative, mse_w (y - target)^2 minus the ARI curve interpolated
at (K - 1) y: d = y - target 143; (2 mse_w) d 145; minus (K-1)(a1 - a0) with
the two ARI values rounded to fp32, 146; dy = that / B, 147.  Backward:
  dW3 = dy h2                147 + 134 + 1 = 282      db3 = dy        147
  dh2 = dy W3 (masked)       148                      db2 = dh2       148
  dW2 = dh2 h1               148 + 69 + 1 = 218
  dh1 = sum of 64 W2 dh2     148 + 1 + 64 = 213       db1 = dh1       213
  dW1 = dh1 xs               213 + 2 + 1 = 216
and the sum over the B rows adds B.  The float64 reference obeys the same
bound with u = 2^-53, so the two may differ by (gamma_k(2^-24) +
gamma_k(2^-53)) times the absolute-value evaluation.

This bound is rigorous but wide for this network: the absolute-value
evaluation lies two to three orders of magnitude above the gradient itself
(cancellation inside each row's dot products), so it catches gross mistakes
only.  The parity tests therefore also apply `empirical_tolerance`, a much
tighter tolerance that is not an a priori bound: its size was set against
measurements, and the CPU pins check that it holds for an independent fp32
evaluation with room to spare and that it rejects a feature scale off by
3 parts in 10^4 or a feature mean off by 10^-4, which the a priori bound
lets through.

The ReLU masks are not polynomial: the backward bound holds where both sides
take the same mask, which is certain when every pre-activation exceeds its own
error bound in magnitude (`rows_with_clear_masks`).  The forward bound needs no
such condition, since ReLU moves no value by more than its argument's error:
there the absolute-value evaluation keeps every unit, masked or not.
"""
import numpy as np

from oracle import mlp

U32 = 2.0 ** -24
U64 = 2.0 ** -53

DEPTH_A1 = 69
DEPTH_A2 = 134
DEPTH_Y = 142
# gradient depths per parameter block, before the B-row sum
DEPTH_GRAD = {"W1": 216, "b1": 213, "W2": 218, "b2": 148, "W3": 282, "b3": 147}


def gamma(k, u):
    k = np.asarray(k, np.float64)
    assert np.all(k * u < 0.5)
    return k * u / (1.0 - k * u)


def both(k):
    """Bound factor between an fp32 and an fp64 evaluation of depth k."""
    return gamma(k, U32) + gamma(k, U64)


def _abs_forward(p, mean, std, x, masks=None):
    """Absolute-value evaluation of the forward pass.  With masks (a1 > 0,
    a2 > 0 of the exact network) the ReLU units take them; without, every
    unit is kept."""
    P = mlp.unpack(np.abs(np.asarray(p, np.float64)))
    xs = (np.abs(np.asarray(x, np.float64)) + np.abs(np.asarray(mean, np.float64))) / np.asarray(std, np.float64)
    a1 = xs @ P["W1"].T + P["b1"]
    h1 = a1 if masks is None else a1 * masks[0]
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = a2 if masks is None else a2 * masks[1]
    y = h2 @ P["W3"] + P["b3"][0]
    return xs, a1, h1, a2, h2, y


def forward_bound(p, mean, std, x):
    """Per-row bound on |y_fp32 - y_fp64|."""
    y = _abs_forward(p, mean, std, x)[-1]
    return both(DEPTH_Y) * y


def rows_with_clear_masks(p, mean, std, x):
    """Rows whose every pre-activation is farther from zero than both
    evaluations' error bound (so fp32, fp64 and exact masks agree)."""
    _, (_, a1, _, a2, _) = mlp.forward(p, mean, std, x)
    _, a1t, _, a2t, _, _ = _abs_forward(p, mean, std, x)
    # the reference's own a1, a2 carry an fp64 error: demand the fp32 bound
    # plus twice the fp64 one
    ok1 = np.abs(a1) > (gamma(DEPTH_A1, U32) + 2 * gamma(DEPTH_A1, U64)) * a1t
    ok2 = np.abs(a2) > (gamma(DEPTH_A2, U32) + 2 * gamma(DEPTH_A2, U64)) * a2t
    return ok1.all(1) & ok2.all(1)


def gradient_bound(p, mean, std, x, target, ari=None, mse_w=1.0):
    """Per-parameter bound on |grad_fp32 - grad_fp64| of the mean row loss,
    valid for rows with clear masks (the caller keeps only those)."""
    P = mlp.unpack(np.abs(np.asarray(p, np.float64)))
    _, (_, a1, _, a2, _) = mlp.forward(p, mean, std, x)
    masks = ((a1 > 0).astype(np.float64), (a2 > 0).astype(np.float64))
    xs, _, h1, _, h2, y = _abs_forward(p, mean, std, x, masks)
    B = len(y)
    dl = 2.0 * mse_w * (y + np.abs(np.asarray(target, np.float64)))
    if ari is not None:
        # the slope term's size, whichever segment is taken
        a = np.abs(np.asarray(ari, np.float64))
        K = a.shape[1]
        dl = dl + (K - 1) * 2.0 * a.max(1)
    dy = dl / B
    dh2 = np.outer(dy, P["W3"]) * masks[1]
    dh1 = (dh2 @ P["W2"]) * masks[0]
    g = {"W3": dy @ h2, "b3": np.array([dy.sum()]), "W2": dh2.T @ h1, "b2": dh2.sum(0),
         "W1": dh1.T @ xs, "b1": dh1.sum(0)}
    depth = {k: np.full(np.shape(v), DEPTH_GRAD[k] + B, np.float64) for k, v in g.items()}
    return mlp.pack(g) * both(mlp.pack(depth))


def grid_position_bound(p, mean, std, x, K):
    """Per-row bound on how far the fp32 grid position (K - 1) y of either
    side lies from the exact one: a row farther than this from every grid
    point and from both ends takes the exact segment on both sides."""
    y = mlp.forward(p, mean, std, x)[0]
    return (K - 1) * (forward_bound(p, mean, std, x) + gamma(2, U32) * np.abs(y))


def row_abs_mean(p, mean, std, x, target, ari=None, mse_w=1.0):
    """(1/B) sum over rows of |d loss_r / d p|, from the float64 reference."""
    P, M, S = (np.asarray(v, np.float64) for v in (p, mean, std))
    T = np.asarray(target, np.float64)
    out = np.zeros(mlp.NPAR)
    for r in range(len(x)):
        g, _ = mlp.gradient(P, M, S, x[r:r + 1], T[r:r + 1], None if ari is None else ari[r:r + 1], mse_w)
        out += np.abs(g)
    return out / len(x)


def empirical_tolerance(g_ref, sabs, B):
    """The parity tests' gradient tolerance: 1e-4 relative per entry (with a
    1e-7 floor), plus 4 (B + 8) u times the mean of the rows' absolute
    gradients for cancellation in the batch sum; (B - 1) u would be the
    recursive-summation bound of that sum alone, and the factor 4 with the
    8 extra terms leave room for the rows' own rounding.  Measured, not
    derived: see the module header."""
    return 1e-4 * (np.abs(g_ref) + 1e-3) + 4 * (B + 8) * U32 * sabs
