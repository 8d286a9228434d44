"""Plain NumPy statements of peak finding and of where a segment should peak,
for the peak-finding tests (no GPU, no library code)."""
import numpy as np

SIGMA = {0: 1, 1: -1, 2: 1, 3: -1}


def local_maxima_topk(outs: dict, k: int, radius: int, min_value: float):
    """fht_peaks' definition: strict (2r+1)^2 maxima per quadrant (s wraps,
    t clipped; an equal neighbour earlier in the quadrant's row-major order
    wins), value >= min_value, the k largest by (value desc, flat index asc),
    ordered by the exact values and reported as float32.
    `outs` maps quadrant -> (array W x H, flat offset of its first element)."""
    cands = []
    for q, (J, base) in outs.items():
        W, H = J.shape
        for t in range(W):
            for s in range(H):
                v = J[t, s]
                if v < min_value:
                    continue
                e = t * H + s
                ok = True
                for dt in range(-radius, radius + 1):
                    tt = t + dt
                    if tt < 0 or tt >= W:
                        continue
                    for ds in range(-radius, radius + 1):
                        ss = (s + ds) % H
                        f = tt * H + ss
                        if f == e:
                            continue
                        u = J[tt, ss]
                        if u > v or (u == v and f < e):
                            ok = False
                            break
                    if not ok:
                        break
                if ok:
                    cands.append((float(v), base + e, q, t, s))
    cands.sort(key=lambda c: (-c[0], c[1]))
    return [(float(np.float32(v)), q, t, s) for v, _, q, t, s in cands[:k]], len(cands)


def segment_lines(r0, c0, r1, c1, R, C):
    """(quadrant, t, s) of the ideal line through a segment, in every quadrant
    whose slope range holds it.  Quadrants 0/1 have lanes = rows x and
    positions = columns y with y = s + sigma t x / (R - 1); 2/3 swap roles."""
    dr, dc = r1 - r0, c1 - c0
    res = []
    if dr != 0 and abs(dc) <= abs(dr):
        m = dc / dr
        sig = 1 if m >= 0 else -1
        t = abs(m) * (R - 1)
        s = (c0 - sig * r0 * abs(m)) % C
        res.append((0 if sig > 0 else 1, t, s, C))
    if dc != 0 and abs(dr) <= abs(dc):
        m = dr / dc
        sig = 1 if m >= 0 else -1
        t = abs(m) * (C - 1)
        s = (r0 - sig * c0 * abs(m)) % R
        res.append((2 if sig > 0 else 3, t, s, R))
    return res


def matches(peak, line, dt_tol=3.0, ds_tol=4.0):
    q, t, s, H = line
    if peak[1] != q:
        return False
    d = abs(peak[3] - s) % H
    return abs(peak[2] - t) <= dt_tol and min(d, H - d) <= ds_tol
