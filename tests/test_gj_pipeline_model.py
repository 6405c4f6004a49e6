"""Host-side model of the pipelined elimination of the N <= 64 kernels
(gj_inverse_pipe: W waves, wave w owning rows RB w .. RB w + RB - 1 of the
matrix, RB = 64 / W), run over random interleavings of the waves.

Each wave takes the published steps of the earlier blocks on its rows, then
its own block's steps (pivot search on its own row, multipliers and pivot
column published, counter raised), then forms its block's inverse rows from
the recorded steps and takes the later steps on them, each after waiting for
its publication.  The same arithmetic in the order of the one-barrier-per-
step elimination (every step on every row of A below it and on every inverse
row created so far) is the reference.  Claims: every run ends; each row
takes the same steps in the same order, so the inverse rows are the same bit
for bit; the result is the inverse; and with waits that may give up (as one
does after its poll limit) every run still ends with the matrix flagged."""
import numpy as np
import pytest

NP = 64


def _key(re, im, lane, used, n):
    if lane in used or lane >= n:
        return 0
    m2 = np.float64(re * re + im * im)
    hi = int(np.array([m2]).view(np.uint64)[0] >> np.uint64(32))
    return (hi & ~63 & 0xFFFFFFFF) | (63 - lane)


def _step(row_re, row_im, used, n):
    """Pivot column and multipliers of one step from the current pivot row."""
    key = max(_key(row_re[j], row_im[j], j, used, n) for j in range(NP))
    pc = 63 - (key & 63)
    px, py = row_re[pc], row_im[pc]
    inv = 1.0 / (px * px + py * py)
    ipx, ipy = px * inv, -py * inv
    f_re = row_re * ipx - row_im * ipy
    f_im = row_re * ipy + row_im * ipx
    f_re[pc], f_im[pc] = 1.0 - ipx, -ipy
    return pc, f_re, f_im, (key >> 6) == 0


def _apply(z_re, z_im, rows, pc, f_re, f_im):
    """Rows of z take step (pc, f): z <- z - f z[pc], the four real
    multiply-adds of the kernels in their order."""
    if len(rows) == 0:
        return
    zp_re = z_re[rows, pc].copy()[:, None]
    zp_im = z_im[rows, pc].copy()[:, None]
    r = z_re[rows] - f_re * zp_re
    r = r + f_im * zp_im
    i = z_im[rows] - f_re * zp_im
    i = i - f_im * zp_re
    z_re[rows], z_im[rows] = r, i


def _sequential(a_re, a_im, n):
    """One step at a time on every row: rows of A below the pivot row and the
    inverse rows created so far (slot k starts as e_{pc_k} at step k)."""
    z_re, z_im = a_re.copy(), a_im.copy()
    s_re, s_im = np.zeros((NP, NP)), np.zeros((NP, NP))
    piv, used = [], set()
    for k in range(n):
        pc, f_re, f_im, _ = _step(z_re[k], z_im[k], used, n)
        used.add(pc)
        piv.append(pc)
        s_re[k, pc] = 1.0
        _apply(z_re, z_im, list(range(k + 1, NP)), pc, f_re, f_im)
        _apply(s_re, s_im, list(range(k + 1)), pc, f_re, f_im)
    return s_re, s_im, piv


def _pipelined(a_re, a_im, n, W, rng, p_give_up):
    RB = NP // W
    rec = [None] * NP
    piv = [None] * NP
    st = {"cnt": 0, "flag": False}
    s_re, s_im = np.zeros((NP, NP)), np.zeros((NP, NP))

    def wait(k):
        while st["cnt"] <= k:
            if st["flag"] or rng.random() < p_give_up:
                st["flag"] = True
                return False
            yield
        return True

    def record(k):
        if rec[k] is None:  # read after a give-up: whatever the memory holds
            return 0, np.zeros(NP), np.zeros(NP)
        return piv[k], rec[k][0], rec[k][1]

    def wave(w):
        k0 = RB * w
        rows = list(range(k0, k0 + RB))
        za_re, za_im = a_re[rows].copy(), a_im[rows].copy()
        zs_re, zs_im = np.zeros((RB, NP)), np.zeros((RB, NP))
        if k0 < n:
            used = set()
            for k in range(k0):
                yield from wait(k)
                pc, f_re, f_im = record(k)
                used.add(pc)
                _apply(za_re, za_im, list(range(RB)), pc, f_re, f_im)
                yield
            for j in range(RB):
                k = k0 + j
                if k >= n:
                    break
                pc, f_re, f_im, sing = _step(za_re[j], za_im[j], used, n)
                if sing:
                    st["flag"] = True
                used.add(pc)
                rec[k], piv[k] = (f_re, f_im), pc
                st["cnt"] = k + 1
                yield
                _apply(za_re, za_im, list(range(j + 1, RB)), pc, f_re, f_im)
            for j in range(RB):
                k = k0 + j
                if k >= n:
                    break
                pc, f_re, f_im = record(k)
                zs_re[j, pc] = 1.0
                _apply(zs_re, zs_im, list(range(j + 1)), pc, f_re, f_im)
            for k in range(k0 + RB, n):
                yield from wait(k)
                pc, f_re, f_im = record(k)
                _apply(zs_re, zs_im, list(range(RB)), pc, f_re, f_im)
                yield
        s_re[rows], s_im[rows] = zs_re, zs_im

    live = {w: wave(w) for w in range(W)}
    ticks = 0
    while live:
        w = rng.choice(sorted(live))
        try:
            next(live[w])
        except StopIteration:
            del live[w]
        ticks += 1
        assert ticks < 2_000_000, "the waves no longer make progress"
    return s_re, s_im, piv[:n], st["flag"]


def _matrix(n, rng):
    a = np.eye(NP, dtype=np.complex128)
    a[:n, :n] = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 2.0 * np.eye(n)
    return a.real.copy(), a.imag.copy(), a


@pytest.mark.parametrize("W", [4, 8])
@pytest.mark.parametrize("n", [1, 5, 8, 16, 17, 33, 48, 61, 64])
def test_pipelined_elimination_matches_the_sequential_one(W, n):
    rng = np.random.default_rng(1000 * W + n)
    a_re, a_im, a = _matrix(n, rng)
    ref_re, ref_im, ref_piv = _sequential(a_re, a_im, n)
    for seed in range(3):
        s_re, s_im, piv, flag = _pipelined(a_re, a_im, n, W, np.random.default_rng(seed), 0.0)
        assert not flag
        assert piv == ref_piv
        assert np.array_equal(s_re[:n], ref_re[:n]) and np.array_equal(s_im[:n], ref_im[:n])
    # slot s is row pc_s of A^{-1}, its entry of column c in lane pc_c
    s = s_re + 1j * s_im
    t = np.zeros((n, n), dtype=np.complex128)
    for sl in range(n):
        t[piv[sl], :] = s[sl, [piv[c] for c in range(n)]]
    inv = np.linalg.inv(a[:n, :n])
    assert np.abs(t - inv).max() <= 1e-10 * np.abs(inv).max()


@pytest.mark.parametrize("W", [4, 8])
@pytest.mark.parametrize("p_give_up", [0.01, 0.3])
def test_pipelined_elimination_ends_when_waits_give_up(W, p_give_up):
    rng = np.random.default_rng(7)
    a_re, a_im, _ = _matrix(61, rng)
    gave_up = 0
    for seed in range(6):
        _, _, _, flag = _pipelined(a_re, a_im, 61, W, np.random.default_rng(seed), p_give_up)
        gave_up += flag
    assert gave_up > 0
