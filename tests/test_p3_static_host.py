"""Host checks of the static-shape p = 3 passes (fwt.hip, fwt_p3s, P3Groups,
plan_p3s), emulated in Python with the kernels' own index arithmetic:

  * every thread's 3^KT elements (e = tid + k TH, TH = 3^(8 - KT)) sit at
    the global offsets the kernel forms (goff0 + k gstep), each tile element
    is loaded once, and they differ exactly in the KT top row digits of the
    pass (k = j0 + 3 j1 + ..., the order dft3_digits expects);
  * each LDS group step partitions the tile into groups of 3^KG elements
    that differ exactly in the step's digits, in dft3_digits' order;
  * the top digits and the group steps together cover every digit of the pass
    once;
  * the static plan covers the m digits in order with shapes fwt_p3s has, and
    only a strided pass of a single digit is left to the generic pass.
"""
import numpy as np
import pytest

E = 6561
KTS = [(rd, kt) for rd in (2, 3, 4, 5, 6, 8) for kt in (2, 3) if rd >= kt]


def shape(rd, kt):
    th = E // 3 ** kt
    w = 3 ** (8 - rd)
    return th, w, th // w  # TH, W, RSTEP = 3^(rd - kt)


def row_digit(rows, i):
    return (rows // 3 ** i) % 3


@pytest.mark.parametrize("rd,kt", KTS)
def test_load_mapping_and_top_digits(rd, kt):
    TH, w, rstep = shape(rd, kt)
    assert rstep == 3 ** (rd - kt) and TH % w == 0
    tid = np.arange(TH)
    sd0 = 3 ** 9 + 17  # any stride: the offsets must follow it exactly
    goff0 = tid % w + (tid // w) * sd0
    gstep = rstep * sd0
    seen = np.zeros(E, dtype=np.int64)
    rows = []
    for k in range(3 ** kt):
        e = tid + k * TH
        assert np.array_equal(goff0 + k * gstep, e % w + (e // w) * sd0)
        np.add.at(seen, e, 1)
        rows.append(e // w)
    assert np.all(seen == 1)
    rows = np.stack(rows, axis=1)  # [tid][k]
    k = np.arange(3 ** kt)
    for i in range(rd - kt):  # lower row digits equal within a thread
        assert np.all(row_digit(rows, i) == row_digit(rows[:, :1], i))
    for t in range(kt):  # top digit rd - kt + t is digit t of k
        assert np.all(row_digit(rows, rd - kt + t) == (k // 3 ** t) % 3)


def group_steps(rd, kt):
    """(Q, KG) of the LDS steps, as P3Groups unrolls them (LIM = rd - kt)."""
    out, q, lim = [], 0, rd - kt
    while q < lim:
        kg = kt if lim - q >= kt else lim - q
        out.append((q, kg))
        q += kg
    return out


@pytest.mark.parametrize("rd,kt", [c for c in KTS if c[0] > c[1]])
def test_group_steps_partition_the_tile(rd, kt):
    TH, w, rstep = shape(rd, kt)
    tid = np.arange(TH)
    covered = list(range(rd - kt, rd))
    for q, kg in group_steps(rd, kt):
        r = 3 ** kg
        pq = 3 ** q
        stq = w * pq
        gpt = E // r // TH
        c = tid % w
        u0 = tid // w
        cover = np.zeros(E, dtype=np.int64)
        for g in range(gpt):
            u = u0 + g * rstep
            lo, hi = u % pq, u // pq
            base = c + w * (lo + pq * r * hi)
            elems = base[:, None] + np.arange(r)[None, :] * stq
            assert elems.max() < E
            np.add.at(cover, elems.ravel(), 1)
            rows = elems // w
            j = np.arange(r)
            assert np.all(elems % w == (elems % w)[:, :1])
            for i in range(rd):
                dig = row_digit(rows, i)
                if q <= i < q + kg:
                    assert np.all(dig == (j // 3 ** (i - q)) % 3)
                else:
                    assert np.all(dig == dig[:, :1])
        assert np.all(cover == 1), (rd, q)
        covered += list(range(q, q + kg))
    assert sorted(covered) == list(range(rd))


def plan_generic(m):
    """The generic planner for 8-byte elements (fwt.hip, plan): emax 8, rows
    of >= 64 bytes (wpref 2), the rest split evenly into passes of <= 6."""
    emax, wpref = 8, 2
    r1 = min(m, emax)
    out = [(0, r1, 0)]
    rest = m - r1
    if rest > 0:
        cap = emax - min(wpref, r1)
        nstr = (rest + cap - 1) // cap
        d = r1
        for i in range(nstr):
            r = (rest - (d - r1) + (nstr - i) - 1) // (nstr - i)
            out.append((d, r, min(wpref, d)))
            d += r
    return out


def plan_p3s(m):
    return [(d0, r, 8 - r if (d0 > 0 and r >= 2) else wd) for d0, r, wd in plan_generic(m)]


def p3s_shape(d0, r, wdig):
    return (d0 == 0 and r == 8 and wdig == 0) or (d0 >= 8 and 2 <= r <= 6 and wdig == 8 - r)


@pytest.mark.parametrize("m", range(1, 17))
def test_static_plan_covers_the_digits(m):
    done = 0
    for d0, r, wdig in plan_p3s(m):
        assert d0 == done and wdig <= d0
        if m >= 8 and not (d0 > 0 and r == 1):
            assert p3s_shape(d0, r, wdig), (m, d0, r, wdig)
        if p3s_shape(d0, r, wdig):
            assert 3 ** r * 3 ** wdig == E and 3 ** m % E == 0
        done += r
    assert done == m
