"""Host check of the staged projection's window arithmetic (no GPU).

A block of the projection A (8 angles by 64 bins) that stages image rows in
LDS reads, for every lane and row it walks, the three columns floor(e) + 1,
+2, +3 of the padded row at window slots floor(e) + kTomoPad + 1 - pb, where
pb is the chunk's window base (a float32 lower bound of the block's leftmost
column over the chunk's 16 rows, rounded down to a multiple of 4) and e the
lane's 32.32 fixed-point hat position.  The kernel stages a block only when
the spread of its hats over a row stays below kProjMaxSpread; this test
re-does that decision and the index arithmetic on the host, exactly for the
fixed-point part and in float32 for the base, and requires every slot to lie
in the 256-column window, over geometries beyond those the GPU tests run.
(The same arithmetic in the kernel is what tests/test_gpu_tomo.py checks bit
for bit against the unstaged gather.)
"""
import numpy as np
import pytest

K_PAD = 104
K_WIN = 256
K_CHUNK = 16
K_ANGLES = 8
K_SPREAD = 208.0
FX = 4294967296.0


def f32(x):
    return np.float32(x)


def fma32(a, b, c):
    # float32 fused multiply-add: the float32 product is exact in float64
    return np.float32(np.float64(np.float32(a)) * np.float64(np.float32(b)) + np.float64(np.float32(c)))


def angle(ny, nx, na, nd, k, i0w):
    c, s = np.cos(np.pi * k / na), np.sin(np.pi * k / na)
    xmaj = abs(c) >= abs(s)
    al, be = (c, s) if xmaj else (s, c)
    nq, nj = (ny, nx) if xmaj else (nx, ny)
    rr = 1.0 / abs(al)
    m = -be / al
    cq0 = 0.5 - 0.5 * nq
    A = lambda b: (b + 0.5 - 0.5 * nd) / al + 0.5 * (nj - 1)
    Af, Al = A(i0w), A(i0w + 63)
    Alo, Ahi = min(Af, Al), max(Af, Al)
    lo_j, hi_j = -rr, (nj - 1) + rr
    ql, qh = 0, nq - 1
    if m == 0.0:
        if not (Ahi > lo_j and Alo < hi_j):
            qh = -1
    else:
        c1, c2 = (lo_j - Ahi) / m, (hi_j - Alo) / m
        cmin, cmax = min(c1, c2), max(c1, c2)
        ql = int(max(np.floor(cmin - cq0) - 1.0, 0.0))
        qh = int(min(np.ceil(cmax - cq0) + 1.0, nq - 1))
    return dict(xmaj=xmaj, al=al, m=m, rr=rr, cq0=cq0, ql=ql, qh=qh,
                elo=Alo - rr, ehi=Ahi - rr, A=A, nj=nj)


def check_block(ny, nx, na, nd, g0, i0w):
    """Returns (staged, worst slot low, worst slot high) for one block."""
    angs = [angle(ny, nx, na, nd, min(g0 + j, na - 1), i0w) for j in range(K_ANGLES)]
    inc = [g0 + j < na and angs[j]["qh"] >= angs[j]["ql"] for j in range(K_ANGLES)]
    if not any(inc):
        return False, None, None
    same = len({a["xmaj"] for a in angs}) == 1
    Q0 = min(a["ql"] for a, i in zip(angs, inc) if i)
    Q1 = max(a["qh"] for a, i in zip(angs, inc) if i)

    def spread(q):
        lo = min(a["elo"] + a["m"] * (q + a["cq0"]) for a, i in zip(angs, inc) if i)
        hi = max(a["ehi"] + a["m"] * (q + a["cq0"]) for a, i in zip(angs, inc) if i)
        return hi - lo
    if not (same and max(spread(Q0), spread(Q1)) < K_SPREAD):
        return False, None, None
    lanes = np.arange(64)
    worst_lo, worst_hi = 10 ** 9, -10 ** 9
    for ch0 in range(Q0, Q1 + 1, K_CHUNK):
        # the chunk's base, in float32 as the kernel forms it
        c0 = f32(f32(ch0) + f32(angs[0]["cq0"]))
        vals = []
        for a, i in zip(angs, inc):
            if not i:
                continue
            cq0 = f32(a["cq0"])
            c0 = np.float32(np.float32(ch0) + cq0)
            c1 = np.float32(c0 + np.float32(K_CHUNK - 1))
            vals.append(min(fma32(a["m"], c0, a["elo"]), fma32(a["m"], c1, a["elo"])))
        pb = (int(np.floor(min(vals))) + K_PAD - 1) & ~3
        for j, (a, i) in enumerate(zip(angs, inc)):
            if not i:
                continue
            rows = [q for q in (ch0, min(ch0 + K_CHUNK - 1, Q1)) if a["ql"] <= q <= a["qh"]]
            if not rows:
                continue
            e0 = a["A"](i0w + lanes) + a["m"] * a["cq0"] - a["rr"]
            dE = int(np.rint(a["m"] * FX))
            E0 = np.array([int(np.rint(v * FX)) for v in e0], dtype=object) + a["ql"] * dE
            for q in rows:
                E = E0 + (q - a["ql"]) * dE
                hi = np.array([int(v) >> 32 for v in E])
                slot = hi + K_PAD + 1 - pb
                worst_lo = min(worst_lo, int(slot.min()))
                worst_hi = max(worst_hi, int(slot.max()) + 2)
    return True, worst_lo, worst_hi


GEOMS = [(2048, 2048, 1000, 2048), (512, 300, 37, 700), (300, 200, 100, 400),
         (1024, 768, 360, 1400), (64, 2000, 90, 300), (4096, 4096, 720, 5800),
         (33, 129, 70, 150), (200, 200, 400, 300)]


@pytest.mark.parametrize("ny,nx,na,nd", GEOMS)
def test_staged_windows_hold_every_tap(ny, nx, na, nd):
    rng = np.random.default_rng(ny * 7 + nx)
    ngroups = (na + K_ANGLES - 1) // K_ANGLES
    nchunks = (nd + 63) // 64
    blocks = [(g, b) for g in range(ngroups) for b in range(nchunks)]
    if len(blocks) > 60:
        # the diagonal groups, the detector's ends, and a random sample
        diag = {int(round(na / 4 / K_ANGLES)), int(round(3 * na / 4 / K_ANGLES))}
        pick = [(g, b) for (g, b) in blocks
                if g in diag or g == 0 or b in (0, nchunks - 1, nchunks // 2)]
        idx = rng.choice(len(blocks), size=40, replace=False)
        blocks = sorted(set(pick[:80]) | {blocks[i] for i in idx})
    staged = 0
    for g, b in blocks:
        st, lo, hi = check_block(ny, nx, na, nd, g * K_ANGLES, b * 64)
        if st:
            staged += 1
            assert lo >= 0 and hi < K_WIN, (g, b, lo, hi)
    assert staged > 0
