"""Host-side model of the two-step kernel's schedule (step2_kernel in
lb_device.hip), checked on the CPU.

The kernel marches a chunk along y; per iteration k the first step's stages
A1, B1, C1, D1 work on pipeline rows k, k-1, k-2, k-3 and the second step's
A2, B2, C2, D2 on rows k-9 .. k-12 (relative to the first step's first output
row). Intermediate values live in rings indexed by row mod ring size. These
tests replay that integer logic for many chunk shapes and check

* that every ring read of a valid stage finds the row it needs (or, at a
  wall, the row whose mirror image stands in for the missing ghost row), and
  that the second step's outputs are exactly the chunk's rows;
* that every cross-lane ring access (LDS) is separated from the conflicting
  write by a barrier, with barriers after phases 1, 2 and 3 only (and that
  dropping one of them is caught)."""
import itertools

import pytest

# ---- row schedule ----------------------------------------------------------


def _regions(Ly, periodic, y0, y1, d):
    """The kernel's S1 / S2 / E2 / stage ranges for a chunk [y0, y1), march d."""
    if d > 0:
        S2, E2 = y0 - 3, y1 + 2
        ws = we = False
        if not periodic:
            S2, E2 = max(S2, 0), min(E2, Ly - 1)
            ws, we = S2 == 0, E2 == Ly - 1
        first, last = y0, y1 - 1
    else:
        S2, E2 = y1 + 2, y0 - 3
        ws = we = False
        if not periodic:
            S2, E2 = min(S2, Ly - 1), max(E2, 0)
            ws, we = S2 == Ly - 1, E2 == 0
        first, last = y1 - 1, y0
    S1 = S2 if ws else S2 - d
    E1 = E2 if we else E2 + d
    rel = lambda y: d * (y - S1)  # noqa: E731
    r2s, r2e = rel(S2), rel(E2)
    return dict(S1=S1, K1=rel(E1) + 1 + 6, a0=S1 - 3 * d, ws=ws, we=we, r2s=r2s, r2e=r2e,
                rbs=r2s + (0 if ws else 1), rbe=r2e - (0 if we else 1),
                rcs=r2s + (0 if ws else 2), rce=r2e - (0 if we else 2),
                rds=rel(first), rde=rel(last), K=rel(last) + 13)


def _replay(Ly, periodic, y0, y1, d, a2_lag=9):
    g = _regions(Ly, periodic, y0, y1, d)
    S1, K1, a0 = g["S1"], g["K1"], g["a0"]
    same = (lambda u, v: (u - v) % Ly == 0) if periodic else (lambda u, v: u == v)  # noqa: E731
    n1, lp1, j1, O = {}, {}, {}, {}
    n2, lp2, j2 = {}, {}, {}
    outs = []
    for k in range(((g["K"] + 7) // 8) * 8):
        s = k % 8
        a = a0 + d * k
        row2 = lambda lag: S1 + d * (k - lag)  # noqa: E731
        # phase 1: A1 on row a, A2 on relative row k-9 from ring rows k-10 .. k-8
        if k < K1:
            n1[s] = a
        r = k - a2_lag
        if g["r2s"] <= r <= g["r2e"]:
            y = row2(a2_lag)
            lo = not periodic and y == 0
            hi = not periodic and y == Ly - 1
            # slot = row mod 4: with lag 9 these are slots s+2, s+3, s (mod 4)
            behind, centre, ahead = (O.get((k - a2_lag + o) & 3) for o in (-1, 0, 1))
            assert same(centre, y)
            south, north = (behind, ahead) if d > 0 else (ahead, behind)
            if not lo:
                assert same(south, y - 1), ("A2 south", k)
            if not hi:
                assert same(north, y + 1), ("A2 north", k)
            n2[(s + 7) & 7] = y
        # phase 2: B1 on row a - d, B2 on relative row k-10
        if 2 <= k < K1:
            assert [n1[(s + 6) & 7], n1[(s + 7) & 7], n1[s]] == [a - 2 * d, a - d, a]
            lp1[(s + 3) & 3] = a - d
        r = k - 10
        if g["rbs"] <= r <= g["rbe"]:
            y = row2(10)
            assert n2.get((s + 6) & 7) == y
            if not (g["ws"] and r == g["r2s"]):
                assert n2.get((s + 5) & 7) == y - d, ("B2 behind", k)
            if not (g["we"] and r == g["r2e"]):
                assert n2.get((s + 7) & 7) == y + d, ("B2 ahead", k)
            lp2[(s + 2) & 3] = y
        # phase 3: C1 on row a - 2d, C2 on relative row k-11
        if 4 <= k < K1:
            assert [lp1[(s + 1) & 3], lp1[(s + 2) & 3], lp1[(s + 3) & 3]] == \
                [a - 3 * d, a - 2 * d, a - d]
            j1[(s + 2) & 3] = a - 2 * d
        r = k - 11
        if g["rcs"] <= r <= g["rce"]:
            y = row2(11)
            assert lp2.get((s + 1) & 3) == y and n2.get((s + 5) & 7) == y
            if not (g["ws"] and r == g["r2s"]):
                assert lp2.get(s & 3) == y - d, ("C2 behind", k)
            if not (g["we"] and r == g["r2e"]):
                assert lp2.get((s + 2) & 3) == y + d, ("C2 ahead", k)
            j2[(s + 1) & 3] = y
        # phase 4: D1 on row a - 3d into the ring, D2 on relative row k-12
        if 6 <= k < K1:
            dd = a - 3 * d
            assert [j1[s & 3], j1[(s + 1) & 3], j1[(s + 2) & 3]] == [dd - d, dd, dd + d]
            assert n1[(s + 5) & 7] == dd
            assert periodic or 0 <= dd < Ly
            O[(s + 2) & 3] = dd
        r = k - 12
        if g["rds"] <= r <= g["rde"]:
            y = row2(12)
            assert n2.get((s + 4) & 7) == y and j2.get(s & 3) == y
            if not (g["ws"] and r == g["r2s"]):
                assert j2.get((s + 3) & 3) == y - d and n2.get((s + 3) & 7) == y - d
            if not (g["we"] and r == g["r2e"]):
                assert j2.get((s + 1) & 3) == y + d and n2.get((s + 5) & 7) == y + d
            outs.append(y)
    assert sorted(outs) == list(range(y0, y1))
    if g["ws"]:
        assert g["S1"] in (0, Ly - 1)


def _chunks(Ly, rows):
    rows = max(min(rows, Ly), min(8, Ly))
    return [(y0, min(Ly, y0 + rows)) for y0 in range(0, Ly, rows)]


@pytest.mark.parametrize("periodic", [False, True])
def test_every_ring_read_finds_its_row(periodic):
    n = 0
    for Ly in (4, 5, 8, 9, 16, 33, 64, 138, 300):
        for rows in (1, 3, 8, 9, 17, 33, 152, Ly):
            for (y0, y1), d in itertools.product(_chunks(Ly, rows), (1, -1)):
                _replay(Ly, periodic, y0, y1, d)
                n += 1
    assert n > 500


def test_a_too_short_lag_is_caught():
    # the model is not vacuous: with the second step 7 rows behind, its pull
    # would need the ring row the first step writes later in the same iteration
    with pytest.raises(AssertionError):
        _replay(64, False, 8, 40, 1, a2_lag=7)


# ---- barrier hazards ------------------------------------------------------


def _accesses(k):
    """(phase, ring, slot, 'r' | 'w') of the LDS rings at iteration k."""
    s = k % 8
    L = [(1, "n1", s, "w")]
    L += [(2, "n1", x, "r") for x in ((s + 6) & 7, (s + 7) & 7, s)] + [(2, "LP1", (s + 3) & 3, "w")]
    L += [(3, "LP1", x, "r") for x in ((s + 1) & 3, (s + 2) & 3, (s + 3) & 3)]
    L += [(3, "n1", (s + 6) & 7, "r"), (3, "J1", (s + 2) & 3, "w")]
    L += [(4, "n1", x, "r") for x in ((s + 4) & 7, (s + 5) & 7, (s + 6) & 7)]
    L += [(4, "J1", x, "r") for x in (s & 3, (s + 1) & 3, (s + 2) & 3)] + [(4, "O", (s + 2) & 3, "w")]
    L += [(1, "O", x, "r") for x in ((s + 2) & 3, (s + 3) & 3, s & 3)] + [(1, "n2", (s + 7) & 7, "w")]
    L += [(2, "n2", x, "r") for x in ((s + 5) & 7, (s + 6) & 7, (s + 7) & 7)] + [(2, "LP2", (s + 2) & 3, "w")]
    L += [(3, "LP2", x, "r") for x in (s & 3, (s + 1) & 3, (s + 2) & 3)]
    L += [(3, "n2", (s + 5) & 7, "r"), (3, "J2", (s + 1) & 3, "w")]
    L += [(4, "n2", x, "r") for x in ((s + 3) & 7, (s + 4) & 7, (s + 5) & 7)]
    L += [(4, "J2", x, "r") for x in ((s + 3) & 3, s & 3, (s + 1) & 3)]
    return sorted(L, key=lambda e: e[0])


def _hazards(barriers_after):
    # time t = 4 k + phase (phase 1..4); a barrier after phase p of iteration k
    # lies between t = 4 k + p and t + 1
    def separated(t0, t1):
        return any((x - 1) % 4 + 1 in barriers_after for x in range(t0, t1))
    last_w, reads, bad = {}, {}, 0
    for k in range(64):
        for ph, ring, slot, rw in _accesses(k):
            key, now = (ring, slot), 4 * k + ph
            if rw == "r":
                if key in last_w and not separated(last_w[key], now):
                    bad += 1
                reads.setdefault(key, []).append(now)
            else:
                bad += sum(1 for r in reads.get(key, []) if r == now or not separated(r, now))
                reads[key] = []
                last_w[key] = now
    return bad


def test_three_barriers_per_iteration_suffice():
    assert _hazards({1, 2, 3}) == 0


@pytest.mark.parametrize("dropped", [1, 2, 3])
def test_each_barrier_is_needed(dropped):
    assert _hazards({1, 2, 3} - {dropped}) > 0


# ---- interior chunks on lattices with walls ----------------------------------


def _inner(Ly, y0, y1):
    # the kernel's rule (step2_kernel): such a chunk takes the body compiled
    # as if periodic
    return y0 >= 8 and y1 <= Ly - 8


def _stage_rows(g, d):
    """Every row a valid stage of the chunk touches: the first step's
    pipeline rows and their pull neighbours, the second step's rows."""
    S1, K1, a0 = g["S1"], g["K1"], g["a0"]
    rows = set()
    for k in range(K1):
        a = a0 + d * k
        rows.update((a - 1, a, a + 1))
    for r in range(g["r2s"], g["r2e"] + 1):
        rows.add(S1 + d * r)
    return rows


@pytest.mark.parametrize("Ly", [16, 17, 40, 64, 2048])
def test_inner_chunks_see_no_wall_row(Ly):
    # For a chunk the rule calls inner, the walls and the periodic reading
    # give the same schedule (no clipping at a wall, no mirrored row), and
    # every row its valid stages touch lies in 0 .. Ly - 1 with the first
    # step's pipeline in 1 .. Ly - 2: no wall or ghost row, so the wall-free
    # body computes what the general one does. The rule is tight: a chunk
    # starting one row higher reaches the wall row.
    seen = 0
    for y0 in range(0, Ly):
        for h in (1, 8, 9, 24, 144):
            y1 = min(Ly, y0 + h)
            for d in (1, -1):
                gw = _regions(Ly, False, y0, y1, d)
                if not _inner(Ly, y0, y1):
                    continue
                seen += 1
                gp = _regions(Ly, True, y0, y1, d)
                assert gw == gp, (y0, y1, d)
                rows = _stage_rows(gw, d)
                assert min(rows) >= 0 and max(rows) <= Ly - 1, (y0, y1, d)
                pipe = [gw["a0"] + d * k for k in range(gw["K1"])]
                assert min(pipe) >= 1 and max(pipe) <= Ly - 2, (y0, y1, d)
    if Ly >= 17:
        assert seen > 0
    # tightness: y0 = 7 puts the wall row 0 into the pipeline
    if Ly >= 24:
        g = _regions(Ly, False, 7, 16, 1)
        assert min(g["a0"] + k for k in range(g["K1"])) == 0
