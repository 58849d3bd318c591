"""FP64 numpy oracle of the learned corrector network (test infrastructure).

TEST INFRASTRUCTURE ONLY: used by tests/ and never by the product path; it
shares no code with the HIP kernels.

The corrector is a 4-layer 3x3 convolutional network with circular (periodic)
padding, 3 -> 32 -> 32 -> 32 -> 2 channels, ReLU after the first three layers,
trained with a mean-squared error and Adam.  The paper itself has no learned
component: this network only corrects a coarse split step towards the fine
one, and the plain fine-step solver stays the reference for its error.

Conventions (shared with the C ABI's flat parameter vector):
  * images are [B, H, W, C] (channels last);
  * layer l has weights w[tap, cout, cin] with tap = 3*dy + dx, dy, dx in
    {0,1,2} meaning offsets (dy-1, dx-1): out[y, x] += in[y+dy-1, x+dx-1] w;
  * the flat vector is, per layer in order, w (9*cout*cin values) then the
    bias (cout values): 864+32 + 9216+32 + 9216+32 + 576+2 = 19970 values.
"""
import numpy as np

LAYERS = [(3, 32, True), (32, 32, True), (32, 32, True), (32, 2, False)]   # (cin, cout, relu)
NPARAMS = sum(9 * ci * co + co for ci, co, _ in LAYERS)


def unflatten(theta):
    """Flat parameter vector -> list of (w[9, cout, cin], b[cout])."""
    theta = np.asarray(theta, dtype=np.float64)
    out, off = [], 0
    for ci, co, _ in LAYERS:
        w = theta[off:off + 9 * co * ci].reshape(9, co, ci)
        off += 9 * co * ci
        b = theta[off:off + co]
        off += co
        out.append((w, b))
    assert off == theta.size == NPARAMS
    return out


def flatten(params):
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in params])


def shifted(x, dy, dx):
    """x[:, y+dy, x+dx, :] with periodic wrap."""
    return np.roll(np.roll(x, -dy, axis=1), -dx, axis=2)


def conv(x, w, b):
    """Circular 3x3 cross-correlation: out = sum_tap shift(x, tap) @ w[tap].T + b."""
    out = np.zeros(x.shape[:3] + (w.shape[1],))
    for tap in range(9):
        dy, dx = tap // 3 - 1, tap % 3 - 1
        out += shifted(x, dy, dx) @ w[tap].T
    return out + b


def conv_direct(x, w, b):
    """The same convolution as explicit loops over pixels (pin for conv)."""
    B, H, W, _ = x.shape
    co = w.shape[1]
    out = np.zeros((B, H, W, co))
    for n in range(B):
        for y in range(H):
            for xx in range(W):
                acc = b.astype(np.float64).copy()
                for tap in range(9):
                    dy, dx = tap // 3 - 1, tap % 3 - 1
                    acc += w[tap] @ x[n, (y + dy) % H, (xx + dx) % W]
                out[n, y, xx] = acc
    return out


def forward(x, theta):
    """Returns the output and every layer's input (for backprop)."""
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for (w, b), (_, _, relu) in zip(unflatten(theta), LAYERS):
        h = conv(h, w, b)
        if relu:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def mse(out, target):
    return float(np.mean((out - target) ** 2))


def backward(x, theta, target):
    """Loss and gradient of the MSE w.r.t. the flat parameters."""
    out, acts = forward(x, theta)
    params = unflatten(theta)
    g = 2.0 * (out - target) / out.size
    grads = [None] * len(LAYERS)
    for li in range(len(LAYERS) - 1, -1, -1):
        w, b = params[li]
        xin, yout = acts[li], acts[li + 1]
        if LAYERS[li][2]:
            g = g * (yout > 0)
        gw = np.zeros_like(w)
        for tap in range(9):
            dy, dx = tap // 3 - 1, tap % 3 - 1
            xs = shifted(xin, dy, dx)
            gw[tap] = np.einsum("bhwo,bhwi->oi", g, xs)
        gb = g.sum(axis=(0, 1, 2))
        grads[li] = (gw, gb)
        if li > 0:
            gx = np.zeros_like(xin)
            for tap in range(9):
                dy, dx = tap // 3 - 1, tap % 3 - 1
                gx += shifted(g @ w[tap], -dy, -dx)
            g = gx
    return mse(out, target), flatten(grads)


def adam(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed, scale=1.0):
    """He-style random initialisation (seeded), zero biases."""
    rng = np.random.default_rng(seed)
    params = []
    for ci, co, _ in LAYERS:
        w = rng.standard_normal((9, co, ci)) * scale * np.sqrt(2.0 / (9 * ci))
        params.append((w, np.zeros(co)))
    return flatten(params)


def bf16_round(a):
    """Round float values to bfloat16 (nearest, ties to even), back as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
