"""Coordinate MLPs of NeuralVDB in float64 (oracle).

Sec. 3.2 defines each network as an MLP from floating-point voxel
coordinates to a value (regression) or a mask state (classification), after
a feature mapping z = gamma(x) (eq. fm, Sec. 3.2.2).  Regressors use the MSE
loss (eq. mse); the level-0 mask classifier uses binary cross-entropy and the
level-1 node classifier a three-class cross-entropy (Sec. 3.3.1).  Training is
Adam with an exponentially decaying learning rate (Sec. 3.2; appendix on
hyper-parameters: decay 0.975 every 100 epochs, lr 1e-3).

Readings taken where the paper is silent:
  * architecture "H x W": H hidden layers of width W with ReLU, then an
    identity (linear) head; the first layer consumes the 2m mapped features
    only (no raw xyz).  The closed-form parameter count below reproduces the
    totals printed in the results tables under exactly this reading.
  * feature mapping: gamma(x) = [cos(2 pi B x) ; sin(2 pi B x)] with B of shape
    (m, 3).  Positional encoding with L octaves is the special case whose row
    3k+d is 2^(k-1) e_d, giving cos/sin(2^k pi x_d).
  * hidden activation ReLU, or sin(omega z) on every hidden layer with
    derivative omega cos(omega z) (appendix on activation functions: sin with
    frequency 1.5 to 3 for smooth volumes; the frequency is read as a factor on
    the pre-activation of each hidden layer, the head staying linear);
  * ReLU'(0) = 0; Adam with beta1 0.9, beta2 0.999, eps 1e-8 added outside
    the square root, no weight decay; lr_s = lr0 * 0.975^floor((s-1)/100).
  * per-sample squared error averaged over the batch (the subscript missing
    on f in eq. mse is read as f_i).
"""
import numpy as np


# ----------------------------------------------------------------------------- architecture
class Shapes(list):
    """Weight shapes [(out, in)] of the layers, with the hidden activation:
    omega = 0 for ReLU, omega > 0 for sin(omega z)."""
    omega = 0.0


class Params(list):
    """Layer parameters [(W_l, b_l)], with the hidden activation as in Shapes."""
    omega = 0.0


def layer_shapes(K, W, H, c, omega=0.0):
    """Weight shapes [(out, in)] of an H x W MLP with K inputs and c outputs."""
    s = Shapes([(W, K)] + [(W, W)] * (H - 1) + [(c, W)])
    s.omega = float(omega)
    return s


def activation(z, omega):
    """Hidden activation: ReLU (omega = 0) or sin(omega z)."""
    return np.maximum(z, 0.0) if omega == 0 else np.sin(omega * z)


def activation_grad(z, omega):
    """Derivative of the hidden activation at z: 1[z > 0] or omega cos(omega z)."""
    return (z > 0).astype(np.float64) if omega == 0 else omega * np.cos(omega * z)


def param_count(K, W, H, c):
    """P(K, W, H, c) = K W + W + (H-1)(W^2 + W) + W c + c."""
    return K * W + W + (H - 1) * (W * W + W) + W * c + c


def unflatten(theta, shapes):
    """Canonical flat layout W1, b1, W2, b2, ... with W_l row-major [out][in]."""
    theta = np.asarray(theta, dtype=np.float64)
    params, o = Params(), 0
    params.omega = getattr(shapes, "omega", 0.0)
    for (n_out, n_in) in shapes:
        Wl = theta[o:o + n_out * n_in].reshape(n_out, n_in); o += n_out * n_in
        bl = theta[o:o + n_out]; o += n_out
        params.append((Wl, bl))
    assert o == theta.size, (o, theta.size)
    return params


def flatten(params):
    return np.concatenate([np.concatenate([Wl.reshape(-1), bl.reshape(-1)]) for Wl, bl in params])


# ----------------------------------------------------------------------------- inputs
def normalize_voxel(p, lo, D):
    """Voxel-centre coordinate scaled into [0,1] over a cubic box (Sec. 3.4)."""
    return (np.asarray(p, np.float64) - np.asarray(lo, np.float64) + 0.5) / float(D)


def normalize_leaf_slot(o, lo, D):
    """Centre of the 8^3 leaf whose origin is o, scaled like normalize_voxel."""
    return (np.asarray(o, np.float64) - np.asarray(lo, np.float64) + 4.0) / float(D)


def pe_matrix(L):
    """Positional-encoding frequencies as a B matrix: row 3k+d = 2^(k-1) e_d."""
    B = np.zeros((3 * L, 3))
    for k in range(L):
        for d in range(3):
            B[3 * k + d, d] = 2.0 ** (k - 1)
    return B


def encode(x, B):
    """gamma(x) = [cos(2 pi B x) ; sin(2 pi B x)]  (eq. fm)."""
    a = 2.0 * np.pi * (np.asarray(x, np.float64) @ np.asarray(B, np.float64).T)
    return np.concatenate([np.cos(a), np.sin(a)], axis=1)


# ----------------------------------------------------------------------------- forward
def forward(params, z0):
    """MLP forward: z_l = W_l h_{l-1} + b_l, h_l = act(z_l), identity head.

    Returns the output (n, c) and the cache [h_0, z_1, h_1, ..., z_H, h_H]."""
    omega = getattr(params, "omega", 0.0)
    h = np.asarray(z0, np.float64)
    cache = [h]
    for Wl, bl in params[:-1]:
        z = h @ Wl.T + bl
        h = activation(z, omega)
        cache += [z, h]
    Wo, bo = params[-1]
    return h @ Wo.T + bo, cache


def predict(params, x, B):
    y, _ = forward(params, encode(x, B))
    return y


# ----------------------------------------------------------------------------- losses
def loss_mse(y, t):
    """eq. mse: mean over the batch of (y_i - t_i)^2 (single output)."""
    y = np.asarray(y, np.float64).reshape(-1)
    return float(np.mean((y - np.asarray(t, np.float64).reshape(-1)) ** 2))


def loss_bce(y, t):
    """Binary cross-entropy on logits: max(y,0) - y t + log(1 + e^-|y|), batch mean."""
    y = np.asarray(y, np.float64).reshape(-1)
    t = np.asarray(t, np.float64).reshape(-1)
    return float(np.mean(np.maximum(y, 0) - y * t + np.log1p(np.exp(-np.abs(y)))))


def loss_ce(y, c):
    """Cross-entropy on logits y (n, k) with class labels c: logsumexp(y) - y_c, batch mean."""
    y = np.asarray(y, np.float64)
    m = y.max(axis=1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(y - m).sum(axis=1))
    return float(np.mean(lse - y[np.arange(len(y)), np.asarray(c, np.int64)]))


def sigmoid(y):
    y = np.asarray(y, np.float64)
    e = np.exp(-np.abs(y))
    return np.where(y >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def output_grad(kind, y, t):
    """dL/dy of the batch-mean losses (hand-derived)."""
    y = np.asarray(y, np.float64)
    n = y.shape[0]
    if kind == "mse":
        return 2.0 * (y - np.asarray(t, np.float64).reshape(y.shape)) / n
    if kind == "bce":
        return (sigmoid(y) - np.asarray(t, np.float64).reshape(y.shape)) / n
    if kind == "ce":
        m = y.max(axis=1, keepdims=True)
        e = np.exp(y - m)
        p = e / e.sum(axis=1, keepdims=True)
        p[np.arange(n), np.asarray(t, np.int64)] -= 1.0
        return p / n
    raise ValueError(kind)


def loss(kind, y, t):
    return {"mse": loss_mse, "bce": loss_bce, "ce": loss_ce}[kind](y, t)


# ----------------------------------------------------------------------------- backward
def backward(params, cache, gy):
    """Hand-derived backward pass.

    For the head and each hidden layer l (top down):
      dW_l = sum_b g_l h_{l-1}^T,  db_l = sum_b g_l,
      g_{l-1} = (W_l^T g_l) * act'(z_{l-1}),
    stopping at the mapped features (no gradient into gamma).
    Returns [(dW_l, db_l)] in layer order."""
    H = len(params) - 1
    omega = getattr(params, "omega", 0.0)
    g = np.asarray(gy, np.float64)
    grads = [None] * (H + 1)
    for l in range(H, -1, -1):
        Wl, _ = params[l]
        h_in = cache[2 * l]                  # h_{l} in 0-based layer numbering (h_0 = gamma)
        grads[l] = (g.T @ h_in, g.sum(axis=0))
        if l > 0:
            z_prev = cache[2 * l - 1]
            g = (g @ Wl) * activation_grad(z_prev, omega)
    return grads


# ----------------------------------------------------------------------------- optimiser
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def lr_at(step, lr0, decay=0.975, interval=100):
    """Staircase exponential decay, step counted from 1."""
    return lr0 * decay ** ((step - 1) // interval)


def adam_step(theta, g, m, v, step, lr, b1=ADAM_B1, b2=ADAM_B2, eps=ADAM_EPS):
    """One bias-corrected Adam update (kingma2014adam); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
