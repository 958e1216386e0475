"""Fracture-block layout of the local linear solve's preconditioner (a
solver choice: the paper leaves the linear solver open, Section 4.3).  The
library cuts each run of consecutive active rows of one fracture inside a
256-row tile into blocks of whole fracture units (a layered fracture's unit
is one segment's cells over its layers) in about equal parts; the layout is
index work and must match the rule computed here on the host exactly."""
import numpy as np
import pytest

from fimgen import make_c1, make_small_c2, make_small_c3

pytestmark = pytest.mark.gpu

TILE = 256
CAP = {1: 64, 2: 20, 3: 21}   # cells per block at most, by block size b


def _frac_id(model):
    f = np.full(model.n, -1, np.int64)
    f[model.n_matrix:] = model.grid["fid"]
    return f


def _units(model, cap):
    """Per cell: unit index inside its fracture and units per block."""
    frac = _frac_id(model)
    unit = np.zeros(model.n, np.int64)
    cu = np.zeros(model.n, np.int64)
    ci, cj = np.asarray(model.conn_i), np.asarray(model.conn_j)
    ulen = np.zeros(model.n, np.int64)
    pos = np.zeros(model.n, np.int64)
    for f in np.unique(frac[frac >= 0]):
        cells = np.nonzero(frac == f)[0]
        pos[cells] = np.arange(cells.size)
        inside = (frac[ci] == f) & (frac[cj] == f)
        bw = int(np.abs(pos[ci[inside]] - pos[cj[inside]]).max()) if inside.any() else 0
        u = bw if 1 <= bw <= cap else 1
        unit[cells] = pos[cells] // u
        cu[cells] = cap // u
        ulen[cells] = u
    return frac, unit, cu, ulen, pos


def _expected(model, l2g, b):
    cap = CAP[b]
    frac, unit, cu, _, _ = _units(model, cap)
    n_a = l2g.size
    start = np.arange(n_a)
    rows = np.ones(n_a, np.int64)
    for t0 in range(0, n_a, TILE):
        rr = np.arange(t0, min(t0 + TILE, n_a))
        fr = frac[l2g[rr]]
        i = 0
        while i < rr.size:
            j = i
            while j < rr.size and fr[j] == fr[i]:
                j += 1
            if fr[i] >= 0:
                us = unit[l2g[rr[i:j]]]
                i0 = us[0]
                ru = int(us[-1] - i0 + 1)
                c = int(cu[l2g[rr[i]]])
                nb = -(-ru // c)
                first = [(k * ru) // nb for k in range(nb)]   # first unit of block k
                blk = np.array([max(k for k in range(nb) if first[k] <= iu) for iu in us - i0])
                for k in np.unique(blk):
                    sel = rr[i:j][blk == k]
                    start[sel] = sel[0]
                    rows[sel] = sel.size
            i = j
    return start, rows, frac, cap


def _check(fm, model, act):
    out = fm.inspect_pc_blocks(act)
    l2g = out["l2g"].astype(np.int64)
    if act is None:
        assert out["n_active"] == model.n
    else:
        assert np.array_equal(l2g, np.nonzero(act)[0])
    start, rows, frac, cap = _expected(model, l2g, model.b)
    assert np.array_equal(out["blk_start"], start)
    assert np.array_equal(out["blk_rows"], rows)
    # every multi-row block: one fracture, inside one tile, at most cap rows
    multi = rows > 1
    assert np.all(rows <= cap)
    s = start[multi]
    e = s + rows[multi] - 1
    assert np.all(s // TILE == e // TILE)
    assert np.all(frac[l2g[s]] == frac[l2g[e]])
    assert np.all(frac[l2g[s]] >= 0)
    return int(multi.sum())


def _models():
    return [
        make_c1(),
        make_small_c2(seed=41, nx=30, ny=16, nz=4, nfrac=24, nstage=3),
        make_small_c3(seed=43, nx=24, ny=12, nz=4, nfrac=16, nstage=2),
        make_small_c2(seed=7, nx=40, ny=20, nz=6, nfrac=60, nstage=4),
    ]


@pytest.mark.parametrize("k", range(4))
def test_block_layout_matches_rule(k):
    from paper_2008_01539_amd import FimModel, Options
    model = _models()[k]
    fm = FimModel(model, Options())
    try:
        covered = _check(fm, model, None)
        assert covered > 0
        rng = np.random.default_rng(100 + k)
        for keep in (0.9, 0.6, 0.3):
            act = (rng.random(model.n) < keep).astype(np.uint8)
            _check(fm, model, act)
        # only the fracture cells: runs span several tiles
        act = (_frac_id(model) >= 0).astype(np.uint8)
        _check(fm, model, act)
    finally:
        fm.close()


def test_layered_units_keep_segments_whole():
    """Two-layer fractures (the DFN) numbered segment by segment have unit
    length 2: with all fracture cells active, a block that starts inside a
    tile starts at an even position of its fracture (a whole segment)."""
    from paper_2008_01539_amd import FimModel, Options
    model = make_small_c3(seed=43, nx=24, ny=12, nz=4, nfrac=16, nstage=2)
    frac, _, _, ulen, pos = _units(model, CAP[model.b])
    fm = FimModel(model, Options())
    try:
        out = fm.inspect_pc_blocks((frac >= 0).astype(np.uint8))
    finally:
        fm.close()
    l2g = out["l2g"].astype(np.int64)
    r = np.arange(l2g.size)
    lead = (out["blk_rows"] > 1) & (out["blk_start"] == r) & (r % TILE != 0)
    lead &= ulen[l2g] == 2
    assert lead.sum() > 0
    assert np.all(pos[l2g[lead]] % 2 == 0)
