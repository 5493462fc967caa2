"""Independent restatements used by the oracle's pin tests (CPU only).

These are written from the definitions in App. B of arXiv 2302.09334 and the
readings of the benchmark workloads, with numpy/torch/fractions, and share no
code with the oracle's C implementation beyond calling its already-pinned
random primitives (Philox, Box-Muller).
"""
from fractions import Fraction

import numpy as np

DR = np.array([-1, 1, 0, 0, 0])
DC = np.array([0, 0, 1, -1, 0])


def genome_to_torch(theta, n_in, hd):
    """Split a genome into torch GRUCell tensors (weight_ih 3Hd x in with gate
    blocks r, z, n; weight_hh 3Hd x Hd; bias_ih; bias_hh) plus the head."""
    theta = np.asarray(theta, np.float64)
    o = 0
    wih = theta[o:o + n_in * hd * 3].reshape(n_in, hd, 3); o += n_in * hd * 3
    whh = theta[o:o + hd * hd * 3].reshape(hd, hd, 3); o += hd * hd * 3
    bih = theta[o:o + hd * 3].reshape(hd, 3); o += hd * 3
    bhh = theta[o:o + hd * 3].reshape(hd, 3); o += hd * 3
    wo = theta[o:o + 5 * hd].reshape(5, hd); o += 5 * hd
    bo = theta[o:o + 5]; o += 5
    assert o == theta.size
    weight_ih = np.concatenate([wih[:, :, g].T for g in range(3)], axis=0)
    weight_hh = np.concatenate([whh[:, :, g].T for g in range(3)], axis=0)
    bias_ih = np.concatenate([bih[:, g] for g in range(3)])
    bias_hh = np.concatenate([bhh[:, g] for g in range(3)])
    return weight_ih, weight_hh, bias_ih, bias_hh, wo, bo


def layer_slices(n_in, hd):
    o = 0
    out = {}
    for name, size in (("W_ih", n_in * hd * 3), ("W_hh", hd * hd * 3), ("b_ih", hd * 3),
                       ("b_hh", hd * 3), ("W_o", 5 * hd), ("b_o", 5)):
        out[name] = slice(o, o + size)
        o += size
    return out


def observation(R, occ_mask, r, c, e, E0, rho):
    """Inputs of an agent: resource window, occupancy window (outside = 1),
    energy / E0."""
    H, W = R.shape
    w = 2 * rho + 1
    xr = np.zeros((w, w))
    xo = np.ones((w, w))
    for dy in range(-rho, rho + 1):
        for dx in range(-rho, rho + 1):
            rr, cc = r + dy, c + dx
            if 0 <= rr < H and 0 <= cc < W:
                xr[dy + rho, dx + rho] = R[rr, cc]
                xo[dy + rho, dx + rho] = occ_mask[rr, cc]
    return np.concatenate([xr.ravel(), xo.ravel(), [e / E0]])


def exact_threshold(cfg, row, n, real=False):
    """floor(p * 2^32) with p in exact rational arithmetic from the decimal
    parameters converted to binary (the same doubles the C code starts from).
    With real=True the unfloored rational p * 2^32 is returned."""
    rb, rt = Fraction(cfg["rate_bottom"]), Fraction(cfg["rate_top"])
    rate = rt + (rb - rt) * row / (cfg["H"] - 1)
    rate *= Fraction(cfg["rate_scale"])
    p = rate * n / 24 + Fraction(cfg["spont"])
    if real:
        return p * (1 << 32)
    if p <= 0:
        return 0
    if p >= 1:
        return 1 << 32
    return int(p * (1 << 32))


def neighbour_counts(R):
    """Resources among the 24 cells at Chebyshev distance 1..2 (outside = 0)."""
    H, W = R.shape
    P = np.zeros((H + 4, W + 4), np.int64)
    P[2:-2, 2:-2] = R
    n = np.zeros((H, W), np.int64)
    for dy in range(-2, 3):
        for dx in range(-2, 3):
            if dy or dx:
                n += P[2 + dy:2 + dy + H, 2 + dx:2 + dx + W]
    return n


def moves_by_priority(H, W, pos, act, keys):
    """Move rule restated as a greedy pass in priority order: agents with a
    valid claim (in-grid target empty at the step start) move in increasing
    key order unless an earlier agent already took the cell."""
    occupied = {tuple(p) for p in pos}
    new = [tuple(p) for p in pos]
    taken = set()
    order = np.argsort(np.asarray(keys, dtype=np.uint64), kind="stable")
    for i in order:
        a = act[i]
        if a == 4:
            continue
        t = (pos[i][0] + DR[a], pos[i][1] + DC[a])
        if not (0 <= t[0] < H and 0 <= t[1] < W):
            continue
        if t in occupied or t in taken:
            continue
        taken.add(t)
        new[i] = t
    return new
