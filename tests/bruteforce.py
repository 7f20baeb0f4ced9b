"""Independent brute-force checker for the oracle (pure Python scalar loops).

Written separately from ``oracle/oracle.c`` (different language, different
loop structure: it gathers each output from an explicit list of taps) so that
a mistake in one is not repeated in the other.  Only for tiny shapes.
"""
import math


def conv2d(x, w, stride, pad):
    """x: nested lists [N][C][H][W]; w: [K][C][R][S]; returns [N][K][Ho][Wo]."""
    N, C, H, W = len(x), len(x[0]), len(x[0][0]), len(x[0][0][0])
    K, R, S = len(w), len(w[0][0]), len(w[0][0][0])
    Ho = (H + 2 * pad - R) // stride + 1
    Wo = (W + 2 * pad - S) // stride + 1
    out = []
    for n in range(N):
        plane_k = []
        for k in range(K):
            rows = []
            for i in range(Ho):
                row = []
                for j in range(Wo):
                    taps = []
                    for r in range(R):
                        for s in range(S):
                            yy, xx = i * stride + r - pad, j * stride + s - pad
                            if 0 <= yy < H and 0 <= xx < W:
                                for c in range(C):
                                    taps.append(w[k][c][r][s] * x[n][c][yy][xx])
                    row.append(sum(taps))
                rows.append(row)
            plane_k.append(rows)
        out.append(plane_k)
    return out


def maxpool(x, size, stride):
    N, C, H, W = len(x), len(x[0]), len(x[0][0]), len(x[0][0][0])
    Ho, Wo = -(-H // stride), -(-W // stride)
    off = (size - 1) // 2
    out = []
    for n in range(N):
        out.append([[[max([x[n][c][i * stride - off + u][j * stride - off + v]
                           for u in range(size) for v in range(size)
                           if 0 <= i * stride - off + u < H and 0 <= j * stride - off + v < W]
                          or [-math.inf])
                      for j in range(Wo)] for i in range(Ho)] for c in range(C)])
    return out
