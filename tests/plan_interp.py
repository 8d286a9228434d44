"""CPU interpreter of the library's tile programs (test helper, host logic only).

It executes the planner's tables with the semantics the gfx950 kernel gives
them and checks the invariants the kernel relies on:

* entries cover whole 64-position chunks: load ``lds[d + c] = src[row][(s0 +
  off + c) mod H]``, merge ``lds[d + c] = lds[a + c] + lds[b + c]`` for
  ``c < 64 k``; load-merge (step 1 of a later pass read from the source
  rows) ``lds[d + c] = src[a][(s0 + off + c) mod H] + src[b][(s0 + off + r +
  c) mod H]`` with ``off | r << 16`` in the entry's last field; store ``dst[row][s0 + c] = lds[d + c]`` (``+ lds[b + c]``
  when the header says the stores add the root's last merge) for
  ``c < min(64 k, limit)`` and ``s0 + c < H``; every row an entry names is
  moved by the header's lane base (programs of equal-width roots share
  entries);
* every LDS access stays inside the program's footprint;
* no merge step reads a range another entry of the same step writes;
* every stored value was computed from loaded data only (positions a window
  does not need may hold garbage, but none of it may reach an output);
* every output element is written exactly once per pass.
"""
import numpy as np

import paper_2411_07351_amd as F

CHUNK = 64


def _overlap(r1, r2):
    return r1[0] < r2[1] and r2[0] < r1[1]


def run_plan_tables(plan_handle, img, q, check=True):
    img = np.asarray(img)
    v, mirror = q >> 1, bool(q & 1)
    A = (img if v == 0 else img.T).astype(np.float64 if img.dtype.kind == "f" else np.int64)
    W, H = A.shape
    if mirror:
        A = A[:, (-np.arange(H)) % H]
    src = A
    npass = F.fht_plan_num_passes(plan_handle, v)
    for p in range(npass):
        tb = F.fht_plan_pass_tables(plan_handle, v, p)
        dst = np.zeros_like(src)
        written = np.zeros(src.shape, dtype=np.int64)
        for prog, _, s0, _ in tb["items"]:
            hdr = tb["hdrs"][prog]
            first, nload, nstore, nsteps, lds_n, nops = (int(x) for x in hdr[:6])
            K, store_merge, nlm = int(hdr[26]), bool(hdr[27]), int(hdr[28])
            base = int(hdr[30])  # lanes added to every row the entries name
            if check:
                # programs with merges fold the last one into the stores
                assert store_merge == (int(hdr[7]) > int(hdr[6]))
            assert nops == nload + nlm + nstore + sum(int(c) for c in hdr[8:8 + nsteps])
            assert int(hdr[25]) == tb["s_tile"]
            ops = tb["ops"][first:first + nops].astype(np.int64)
            ops[:nload + nlm, 1] += base
            ops[nload:nload + nlm, 2] += base
            ops[nops - nstore:, 1] += base
            lds = np.zeros(lds_n, dtype=src.dtype)
            valid = np.zeros(lds_n, dtype=bool)
            if check and int(hdr[6]) == 0:
                # first pass: one entry per lane of the root, in lane order
                rows = ops[:nload, 1]
                assert nload <= 64 and (np.diff(rows) == 1).all()
                assert int(hdr[24]) == int((ops[:nload, 2] + CHUNK * ops[:nload, 3]).max())
            for d, row, off, k in ops[:nload]:
                n = CHUNK * int(k)
                if check:
                    assert 1 <= k <= 4 and 0 <= d and d + n <= lds_n and 0 <= row < W and off >= 0
                pos = (s0 + off + np.arange(n)) % H
                lds[d:d + n] = src[row, pos]
                valid[d:d + n] = True
            if check:
                # load-merges only in later passes whose LDS elements are not 4 bytes
                assert nlm == 0 or (int(hdr[6]) > 0 and int(hdr[29]) != 4)
                spans = [(int(d), int(d) + CHUNK * K) for d, _, _, _ in ops[:nload + nlm]]
                for i, a in enumerate(spans):
                    assert 0 <= a[0] and a[1] <= lds_n
                    assert not any(_overlap(a, b) for b in spans[i + 1:]), "loads overlap"
            for d, ra, rb, offs in ops[nload:nload + nlm]:
                offs = int(offs) & 0xFFFFFFFF
                n = CHUNK * K
                if check:
                    assert 0 <= ra < W and 0 <= rb < W
                pa = (s0 + (offs & 0xFFFF) + np.arange(n)) % H
                pb = (s0 + (offs & 0xFFFF) + (offs >> 16) + np.arange(n)) % H
                lds[d:d + n] = src[ra, pa] + src[rb, pb]
                valid[d:d + n] = True
            e = nload + nlm
            for step in range(nsteps):
                cnt = int(hdr[8 + step])
                step_ops = ops[e:e + cnt]
                if check:
                    assert ((step_ops[:, 3] >= 1) & (step_ops[:, 3] <= 4)).all()
                    writes = [(d, d + CHUNK * k) for d, a, b, k in step_ops]
                    reads = [(a, a + CHUNK * k) for d, a, b, k in step_ops] + \
                            [(b, b + CHUNK * k) for d, a, b, k in step_ops]
                    for w in writes:
                        assert w[0] >= 0 and w[1] <= lds_n
                        for r in reads:
                            assert r[0] >= 0 and r[1] <= lds_n
                            assert not _overlap(w, r), "merge step reads what it writes"
                new = []
                for d, a, b, k in step_ops:
                    n = CHUNK * int(k)
                    new.append((d, lds[a:a + n] + lds[b:b + n], valid[a:a + n] & valid[b:b + n]))
                for d, vals, ok in new:
                    lds[d:d + len(vals)] = vals
                    valid[d:d + len(vals)] = ok
                e += cnt
            for d, row, lim, b in ops[e:e + nstore]:
                m = max(0, min(CHUNK * K, int(lim), H - int(s0)))
                vals, ok = lds[d:d + m], valid[d:d + m]
                if check:
                    assert 0 <= d and d + CHUNK * K <= lds_n
                    assert (b >= 0) == store_merge
                if store_merge:
                    if check:
                        assert b + CHUNK * K <= lds_n
                    vals, ok = vals + lds[b:b + m], ok & valid[b:b + m]
                if check:
                    assert ok.all(), "a stored value depends on unloaded data"
                dst[row, s0:s0 + m] = vals
                written[row, s0:s0 + m] += 1
        if check:
            assert (written == 1).all(), f"pass {p} does not write every element exactly once"
        src = dst
    out = src
    if mirror:
        out = out[:, (-np.arange(H)) % H]
    return out
