"""Reference U-Net for the learned initial guess (test infrastructure only).

The learned part is not in the paper; its network is fixed here as a 3D
U-Net on the element grid of the auxiliary mesh.  The
input has one channel per node of an element (the nodal values of rho/s,
s a per-sample scale), the output one channel per node (the nodal values of
v/s).  With channels last, the element-major field order of the library is
exactly the network's [z][y][x][channel] tensor.

Architecture (L levels, C channels, ReLU after every convolution but the last):
    h   = relu(in(x))                              1x1x1, Cin -> C
    for l = 0 .. L-1:
        e_l = relu(enc_l_b(relu(enc_l_a(h))))      3x3x3, C -> C, twice
        if l < L-1: h = relu(down_l(e_l))          3x3x3 stride 2, C -> C
    d = e_{L-1}
    for l = L-2 .. 0:
        u = relu(up_l(upsample2(d)))               nearest x2, then 3x3x3, C -> C
        d = relu(merge_l(concat(u, e_l)))          3x3x3, 2C -> C
    y   = out(d)                                   1x1x1, C -> Cout
Convolutions pad with zeros (padding 1 for 3x3x3); a stride-2 convolution of
an extent n gives ceil(n/2).  Weights of a convolution are W[tap][ci][co] with
tap = (dz*3 + dy)*3 + dx (one tap for 1x1x1), followed by its bias[co]; the
parameter vector is the convolutions in the order above.

Loss: relative A-norm error  ||s y - v*||_A^2 / ||v*||_A^2  with A the SIPDG
matrix of the mesh.  Adam: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
p -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps)  (Kingma & Ba 2015).
"""
import numpy as np


def layer_specs(levels, channels, cin, cout):
    """[(name, ksize, stride, in_ch, out_ch)] in parameter order."""
    C = channels
    specs = [("in", 1, 1, cin, C)]
    for l in range(levels):
        specs += [(f"enc{l}a", 3, 1, C, C), (f"enc{l}b", 3, 1, C, C)]
        if l < levels - 1:
            specs.append((f"down{l}", 3, 2, C, C))
    for l in range(levels - 2, -1, -1):
        specs += [(f"up{l}", 3, 1, C, C), (f"merge{l}", 3, 1, 2 * C, C)]
    specs.append(("out", 1, 1, C, cout))
    return specs


def param_count(specs):
    return sum(k ** 3 * ci * co + co for _, k, _, ci, co in specs)


def unpack(params, specs):
    out, off = {}, 0
    for name, k, s, ci, co in specs:
        nw = k ** 3 * ci * co
        W = params[off:off + nw].reshape(k ** 3, ci, co)
        off += nw
        b = params[off:off + co]
        off += co
        out[name] = (W, b, k, s)
    return out


def conv(x, W, b, k, s):
    """x [B, D, H, Wd, Ci] -> [B, D', H', W', Co]; zero padding (k-1)/2, stride s."""
    B, D, H, Wd, Ci = x.shape
    pad = (k - 1) // 2
    Do, Ho, Wo = (-(-D // s), -(-H // s), -(-Wd // s))
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (pad, pad), (0, 0)))
    y = np.zeros((B, Do, Ho, Wo, W.shape[2]), dtype=x.dtype)
    for dz in range(k):
        for dy in range(k):
            for dx in range(k):
                t = (dz * k + dy) * k + dx
                patch = xp[:, dz:dz + s * (Do - 1) + 1:s, dy:dy + s * (Ho - 1) + 1:s, dx:dx + s * (Wo - 1) + 1:s, :]
                y += patch @ W[t]
    return y + b


def conv_backward(x, W, k, s, dy):
    """Gradients (dx, dW, db) of conv for upstream dy."""
    B, D, H, Wd, Ci = x.shape
    pad = (k - 1) // 2
    Do, Ho, Wo = dy.shape[1:4]
    xp = np.pad(x, ((0, 0), (pad, pad), (pad, pad), (pad, pad), (0, 0)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for dz in range(k):
        for dy_ in range(k):
            for dx in range(k):
                t = (dz * k + dy_) * k + dx
                sl = (slice(None), slice(dz, dz + s * (Do - 1) + 1, s), slice(dy_, dy_ + s * (Ho - 1) + 1, s),
                      slice(dx, dx + s * (Wo - 1) + 1, s), slice(None))
                patch = xp[sl]
                dW[t] = np.einsum("bzyxi,bzyxo->io", patch, dy)
                dxp[sl] += dy @ W[t].T
    dx = dxp[:, pad:pad + D, pad:pad + H, pad:pad + Wd, :]
    db = dy.sum(axis=(0, 1, 2, 3))
    return dx, dW, db


def upsample2(x, shape):
    """Nearest-neighbour x2 upsampling cropped to spatial shape."""
    y = x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)
    return y[:, :shape[0], :shape[1], :shape[2], :]


def upsample2_backward(dy, shape_in):
    B, D, H, W, C = dy.shape
    dx = np.zeros((B,) + tuple(shape_in) + (C,), dtype=dy.dtype)
    for a in range(2):
        for b in range(2):
            for c in range(2):
                part = dy[:, a::2, b::2, c::2, :]
                dx[:, :part.shape[1], :part.shape[2], :part.shape[3], :] += part
    return dx


def forward(params, specs, levels, x):
    """Returns (y, cache)."""
    P = unpack(params, specs)
    cache = {}

    def run(name, inp):
        W, b, k, s = P[name]
        z = conv(inp, W, b, k, s)
        cache[name] = (inp, z)
        return z

    relu = lambda z: np.maximum(z, 0.0)
    h = relu(run("in", x))
    enc = []
    for l in range(levels):
        a = relu(run(f"enc{l}a", h))
        e = relu(run(f"enc{l}b", a))
        enc.append(e)
        if l < levels - 1:
            h = relu(run(f"down{l}", e))
    d = enc[-1]
    for l in range(levels - 2, -1, -1):
        up = upsample2(d, enc[l].shape[1:4])
        cache[f"upsrc{l}"] = d.shape[1:4]
        u = relu(run(f"up{l}", up))
        d = relu(run(f"merge{l}", np.concatenate([u, enc[l]], axis=-1)))
    y = run("out", d)
    return y, cache


def backward(params, specs, levels, cache, dy):
    """Gradient of sum(y * dy) with respect to the parameters (same layout)."""
    P = unpack(params, specs)
    grads = {}

    def back(name, g, relu_after):
        inp, z = cache[name]
        if relu_after:
            g = g * (z > 0)
        W, b, k, s = P[name]
        dx, dW, db = conv_backward(inp, W, k, s, g)
        grads[name] = (dW, db)
        return dx

    g = back("out", dy, False)
    genc = [None] * levels
    for l in range(0, levels - 1):
        gm = back(f"merge{l}", g, True)
        C = gm.shape[-1] // 2
        gu, ge = gm[..., :C], gm[..., C:]
        genc[l] = ge
        gup = back(f"up{l}", gu, True)
        g = upsample2_backward(gup, cache[f"upsrc{l}"])
    # g is now the gradient of d = e_{L-1}
    gh = None
    for l in range(levels - 1, -1, -1):
        ge = g if l == levels - 1 else genc[l] + gdown_to_e
        ga = back(f"enc{l}b", ge, True)
        gh = back(f"enc{l}a", ga, True)
        if l > 0:
            gdown_to_e = back(f"down{l - 1}", gh, True)
    back("in", gh, True)
    flat = []
    for name, *_ in specs:
        dW, db = grads[name]
        flat += [dW.reshape(-1), db]
    return np.concatenate(flat)


def adam(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
