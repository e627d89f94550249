"""Exact rational evaluation of tiny predicate models (pins the fp64 oracle).

Pure-Python loops over ``fractions.Fraction``; written independently of the
oracle (no numpy arithmetic, no im2col, no shared helpers).  fp32 weights and
bf16/fp32 frame values are dyadic rationals, so every quantity below is exact.
"""
from fractions import Fraction as F


def exact_value(x):
    return F(float(x))          # float -> exact dyadic rational


def normalised(v):
    return (v - F(1, 2)) * 4


def mlp_exact(frame, W1, b1, W2, b2):
    """frame: nested [H][W][3] of Fractions (raw values). Returns 10 exact logits."""
    flat = [normalised(frame[y][x][c])
            for y in range(len(frame)) for x in range(len(frame[0])) for c in range(3)]
    h = []
    for j in range(len(b1)):
        s = exact_value(b1[j])
        for i, v in enumerate(flat):
            s += exact_value(W1[i][j]) * v
        h.append(s if s > 0 else F(0))
    z = []
    for c in range(len(b2)):
        s = exact_value(b2[c])
        for j, v in enumerate(h):
            s += exact_value(W2[j][c]) * v
        z.append(s)
    return z


def conv_exact(act, W, b):
    """act: [H][W][C] exact (normalised); W [O][C][3][3]; stride 2, zero pad 1, ReLU."""
    H, Wd, C = len(act), len(act[0]), len(act[0][0])
    Ho, Wo = (H + 1) // 2, (Wd + 1) // 2
    O = len(b)
    out = [[[F(0)] * O for _ in range(Wo)] for _ in range(Ho)]
    for i in range(Ho):
        for j in range(Wo):
            for o in range(O):
                s = exact_value(b[o])
                for c in range(C):
                    for u in range(3):
                        for v in range(3):
                            y, x = 2 * i + u - 1, 2 * j + v - 1
                            if 0 <= y < H and 0 <= x < Wd:
                                s += exact_value(W[o][c][u][v]) * act[y][x][c]
                out[i][j][o] = s if s > 0 else F(0)
    return out


def cnn_exact(frame, convs, Wfc, bfc):
    act = [[[normalised(frame[y][x][c]) for c in range(3)] for x in range(len(frame[0]))]
           for y in range(len(frame))]
    for W, b in convs:
        act = conv_exact(act, W, b)
    H, Wd, C = len(act), len(act[0]), len(act[0][0])
    g = []
    for c in range(C):
        s = F(0)
        for y in range(H):
            for x in range(Wd):
                s += act[y][x][c]
        g.append(s / (H * Wd))
    z = []
    for k in range(len(bfc)):
        s = exact_value(bfc[k])
        for c in range(C):
            s += exact_value(Wfc[c][k]) * g[c]
        z.append(s)
    return z


def margin_exact(z, class_mask):
    inside = [z[c] for c in range(len(z)) if (class_mask >> c) & 1]
    outside = [z[c] for c in range(len(z)) if not (class_mask >> c) & 1]
    if not inside:
        return None, "neg_inf"
    if not outside:
        return None, "pos_inf"
    return max(inside) - max(outside), "finite"
