"""The grouped schedule of the mixed-precision factorization (the look-ahead
and the plain form of mxp_factor_impl in csrc/driver.hip, transcribed step for
step) checked against what right-looking LU without pivoting needs (Sec. II):
every element receives each earlier panel's update exactly once, all before
the FACT or the U12 solve that finalizes it; every update reads operand slots
that the right panel's conversion wrote; and, with two streams, every pair of
accesses to one element from different streams (one of them a write) is
ordered by an event.  A change of the C++ schedule is to be mirrored here."""
import numpy as np
import pytest

def run(n, nb, la, joint=2048, maxg=32, drop_wait=False):
    G = max(1, min(joint // nb, maxg))
    gw = G * nb
    npan = (n + nb - 1) // nb
    clock = {0: np.zeros(2, int), 1: np.zeros(2, int)}  # vector clocks of streams 0 (main) and 1 (panel)
    evs = {}
    last_w = {}   # element -> (stream, clock value at write, op)
    last_r = {}   # element -> list of (stream, clockvalue)
    contrib = {}  # element -> list of panels
    finalized = {}  # element -> done (fact or trsm)
    bufslot = {}  # (q, slot, idx) -> (panel, stream, clk)
    errors = []
    def tick(s):
        clock[s][s] += 1
        return clock[s].copy()
    def hb(a_stream, a_clk, b_stream):  # does op a (on a_stream at a_clk[a_stream]) happen before now on b_stream?
        return clock[b_stream][a_stream] >= a_clk
    def access(s, cells_w, cells_r, tag):
        c = tick(s)
        for e in cells_r:
            if e in last_w:
                ws, wc, wop = last_w[e]
                if ws != s and not hb(ws, wc, s):
                    errors.append(f"race: {tag} reads {e} written by {wop} on stream {ws}")
        for e in cells_w:
            if e in last_w:
                ws, wc, wop = last_w[e]
                if ws != s and not hb(ws, wc, s):
                    errors.append(f"race: {tag} writes {e} written by {wop}")
            for rs, rc in last_r.get(e, []):
                if rs != s and not hb(rs, rc, s):
                    errors.append(f"race: {tag} writes {e} read on stream {rs}")
            last_w[e] = (s, c[s], tag)
            last_r[e] = []
        for e in cells_r:
            last_r.setdefault(e, []).append((s, c[s]))
        return c
    def rng(a, b): return range(max(a, 0), min(b, n))
    def fact(c, w, s):
        cells = [(i, j) for j in rng(c, c + w) for i in rng(c, n)]
        for (i, j) in cells:
            need = set(range(min(i // nb, j // nb)))
            if set(contrib.get((i, j), [])) != need:
                errors.append(f"fact {c}: element {(i, j)} has {sorted(contrib.get((i, j), []))} need {sorted(need)}")
            finalized[(i, j)] = True
        access(s, cells, cells, f"fact{c}")
    def prep(c, q, idx, slot, s, b0):
        rows = [(i, j) for i in rng(c, c + nb) for j in rng(c + nb, n)]
        for (i, j) in rows:
            need = set(range(i // nb))
            if set(contrib.get((i, j), [])) != need:
                errors.append(f"prep {c}: element {(i, j)} has {sorted(contrib.get((i, j), []))} need {sorted(need)}")
            finalized[(i, j)] = True
        l11 = [(i, j) for i in rng(c, c + nb) for j in rng(c, c + nb)]
        l21 = [(i, j) for i in rng(c + nb, n) for j in rng(c, c + nb)]
        clk = access(s, rows, l11 + rows + l21, f"prep{c}")
        for x in range(c + nb, n):
            bufslot[(q, slot, x - b0)] = (c // nb, s, clk[s])
        if c + nb - b0 != idx:
            errors.append(f"prep {c}: idx {idx} != {c + nb - b0}")
    def update(b0, q, i0, ni, j0, nc, K, s, gp0):
        if ni <= 0 or nc <= 0: return
        cells = [(i, j) for i in range(b0 + i0, b0 + i0 + ni) for j in range(b0 + j0, b0 + j0 + nc)]
        if any(i >= n or j >= n for i, j in cells):
            errors.append(f"update out of range {(b0, i0, ni, j0, nc)}")
        # buffer reads
        for slot in range(K // nb):
            for x in list(range(i0, i0 + ni)) + list(range(j0, j0 + nc)):
                v = bufslot.get((q, slot, x))
                if v is None or v[0] != gp0 + slot:
                    errors.append(f"update reads buffer {q} slot {slot} idx {x}: {v} expected panel {gp0 + slot}")
                    break
                ps, pc = v[1], v[2]
                if ps != s and not hb(ps, pc, s):
                    errors.append(f"race on buffer {q} slot {slot}")
                    break
        for (i, j) in cells:
            if finalized.get((i, j)):
                errors.append(f"update of finalized {(i, j)}")
            contrib.setdefault((i, j), []).extend(range(gp0, gp0 + K // nb))
        access(s, cells, cells, f"upd{b0},{i0},{j0}")
    def record(e, s): evs[e] = clock[s].copy()
    def wait(s, e): clock[s] = np.maximum(clock[s], evs[e])
    ST, SP = 0, (1 if la else 0)
    def group_panels(c, q, s, ev):
        b0 = c + nb
        for i in range(G):
            ci = c + i * nb
            if ci >= n: break
            wi = min(n - ci, nb)
            if i > 0:
                if ev: wait(s, 2 * i)
                update(b0, q, ci - b0, n - ci, ci - b0, wi, i * nb, s, c // nb)
                fact(ci, wi, s)
            if ci + wi >= n: break
            if ev and not drop_wait: wait(s, 2 * i + 1)
            if i > 0: update(b0, q, ci - b0, wi, ci + wi - b0, n - ci - wi, i * nb, s, c // nb)
            prep(ci, q, ci + wi - b0, i, s, b0)
    fact(0, min(nb, n), ST)
    cur = 0
    if nb < n: group_panels(0, cur, ST, False)
    c = 0
    while c + gw < n:
        b0, c2 = c + nb, c + gw
        i2, m2 = c2 - b0, n - c2
        w0 = min(m2, nb)
        q = cur if la else 0
        if not la:
            update(b0, 0, i2, m2, i2, m2, gw, ST, c // nb)
            fact(c2, w0, ST)
            if m2 > w0: group_panels(c2, 0, ST, False)
        else:
            done = i2
            i = 0
            while i < G and done < n - b0:
                wi = min(n - b0 - done, nb)
                update(b0, cur, done, n - b0 - done, done, wi, gw, ST, c // nb)
                record(2 * i, ST)
                if i == 0:
                    wait(SP, 0)
                    fact(c2, w0, SP)
                update(b0, cur, done, wi, done + wi, n - b0 - done - wi, gw, ST, c // nb)
                record(2 * i + 1, ST)
                done += wi
                i += 1
            if m2 > w0: group_panels(c2, cur ^ 1, SP, True)
            update(b0, cur, done, n - b0 - done, done, n - b0 - done, gw, ST, c // nb)
            record(99, SP)
            wait(ST, 99)
        cur ^= 1
        c += gw
    # every element finalized (fact for j-panel columns rows >= panel start; prep for row blocks)
    for i in range(n):
        for j in range(n):
            if not finalized.get((i, j)):
                errors.append(f"element {(i, j)} never finalized")
                break
    return errors


@pytest.mark.parametrize("n", [1, 64, 130, 300])
@pytest.mark.parametrize("nb", [64, 128])
@pytest.mark.parametrize("joint", [64, 256])
@pytest.mark.parametrize("la", [False, True])
def test_mxp_group_schedule(n, nb, joint, la):
    assert run(n, nb, la, joint=joint) == []


def test_mxp_group_schedule_catches_a_missing_wait():
    """The checker itself: a look-ahead schedule whose panel stream skips the
    wait for its rows' region must be reported."""
    errs = run(300, 64, True, joint=128, drop_wait=True)
    assert any("race" in e for e in errs)
