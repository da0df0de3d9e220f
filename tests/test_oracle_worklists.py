"""Pins of the oracle's tile support lists and work counts (CPU).

The oracle's ``tile_lists`` is the reference the binning stage is compared
with, and ``work_counts`` gives the roofline's algorithmic work (support
pairs, alpha evaluations up to each pixel's stop, the tile-lockstep count and
the contributing pairs).  Both are pinned here against the independent numpy
brute force (``oracle/brute.py``: its own rotation, covariance and inverse,
every Gaussian evaluated at every pixel centre with no bounding box) and
against identities with the oracle's own render:

* a block's list holds exactly the Gaussians whose clamped alpha reaches
  alpha_min at some pixel centre of the block, in (depth key, index) order
  (Sec. 3.1: Gaussians are blended front to back in depth order);
* pairs = sum of the list lengths; contributing pairs = the sum of the
  render's per-pixel contributor counts and the brute force's count of
  blended (pixel, Gaussian) pairs; alpha evaluations = the brute force's
  per-pixel count of covering Gaussians of the block's list up to and
  including the one that stops the pixel; the lockstep count = block area
  times the longest such prefix, so it is never below the evaluations.
"""
import numpy as np
import pytest

from oracle import brute
from paper_2504_19409_amd import scenegen as sg


def _scenes():
    out = []
    sc, _ = sg.workload_scene("tiny")  # 2,000 Gaussians, 64x48
    out.append(("tiny", sc))
    out.append(("ragged", sg.make_scene(300, 70, 50, 50.0, 50.0, 35.0, 25.0, 3, seed=31)))
    rng = np.random.default_rng(32)
    vm, _ = sg.perturbed_viewmat(rng, sg.identity_viewmat(), 0.1, 10.0)
    out.append(("rotated", sg.make_scene(400, 45, 37, 40.0, 40.0, 22.5, 18.5, 2, seed=32,
                                         viewmat=vm)))
    dense = sg.make_scene(3000, 40, 36, 40.0, 40.0, 20.0, 18.0, 2, seed=33)
    dense.log_scales += 0.8  # large overlapping splats: most pixels saturate and stop
    out.append(("dense", dense))
    return out


SCENES = _scenes()


def _dicts(sc):
    import oracle
    return oracle.scene_dicts(sc)


def _brute_lists(sp, W, H, tile, alpha_min=1 / 255):
    tx, ty = -(-W // tile), -(-H // tile)
    A = sp["alpha"].reshape(-1, H, W)
    lists = []
    for by in range(ty):
        for bx in range(tx):
            blk = A[:, by * tile:(by + 1) * tile, bx * tile:(bx + 1) * tile]
            hit = (blk >= alpha_min).reshape(blk.shape[0], -1).any(axis=1)
            lists.append(np.nonzero(hit)[0])  # positions in blending order
    return lists, tx, ty


def _brute_work(sp, W, H, tile, alpha_min=1 / 255, t_min=1e-4):
    """(pairs, evals, tile_evals, contribs) by brute force."""
    lists, tx, ty = _brute_lists(sp, W, H, tile, alpha_min)
    pairs = sum(len(l) for l in lists)
    evals = tile_evals = contribs = 0
    ys, xs = np.mgrid[0:H, 0:W]
    for t, pos in enumerate(lists):
        by, bx = divmod(t, tx)
        sl = (slice(by * tile, (by + 1) * tile), slice(bx * tile, (bx + 1) * tile))
        px = xs[sl].reshape(-1) + 0.5
        py = ys[sl].reshape(-1) + 0.5
        npx = px.size
        if len(pos) == 0:
            continue
        a = sp["alpha"].reshape(-1, H, W)[pos][:, sl[0], sl[1]].reshape(len(pos), npx)
        cov = ((np.abs(px[None, :] - sp["u"][pos][:, None]) <= sp["rx"][pos][:, None]) &
               (np.abs(py[None, :] - sp["v"][pos][:, None]) <= sp["ry"][pos][:, None]))
        T = np.ones(npx)
        live = np.ones(npx, dtype=bool)
        stop_at = np.full(npx, len(pos))
        ne = np.zeros(npx, dtype=np.int64)
        for j in range(len(pos)):
            ne += (live & cov[j]).astype(np.int64)
            ok = live & cov[j] & (a[j] >= alpha_min)
            Tn = T * (1.0 - a[j])
            stop = ok & (Tn < t_min)
            stop_at[stop] = j + 1
            live &= ~stop
            ok &= ~stop
            contribs += int(ok.sum())
            T = np.where(ok, Tn, T)
        evals += int(ne.sum())
        tile_evals += int(stop_at.max()) * tile * tile
    return pairs, evals, tile_evals, contribs


@pytest.mark.parametrize("name,sc", SCENES, ids=[n for n, _ in SCENES])
@pytest.mark.parametrize("tile", [16, 8, 5])
def test_tile_lists_equal_brute_force(oracle_lib, name, sc, tile):
    p, c = _dicts(sc)
    counts, ids = oracle_lib.tile_lists(p, c, tile=tile)
    sp = brute.splats(p, c)
    lists, tx, ty = _brute_lists(sp, c["width"], c["height"], tile)
    assert counts.shape == (tx * ty,)
    want = [sp["ids"][l] for l in lists]
    assert [int(x) for x in counts] == [len(l) for l in want]
    start = np.concatenate([[0], np.cumsum(counts)])
    for t in range(tx * ty):
        np.testing.assert_array_equal(ids[start[t]:start[t + 1]], want[t], err_msg=f"tile {t}")
    assert counts.sum() > 0


def test_tile_lists_order_is_depth_then_index(oracle_lib):
    # two Gaussians at exactly the same depth key: the lower index comes first,
    # and swapping their depths swaps them
    P = 3
    means = np.array([[0.0, 0.05, -0.05], [0.0, 0.02, 0.01], [2.0, 2.0, 1.5]], np.float32)
    params = dict(means=means, log_scales=np.full((3, P), -2.0, np.float32),
                  quats=np.tile(np.array([[1.0], [0], [0], [0]], np.float32), (1, P)),
                  logit_opacity=np.zeros(P, np.float32), rgb=np.ones((3, P), np.float32),
                  feat=None)
    cam = dict(width=32, height=32, fx=30.0, fy=30.0, cx=16.0, cy=16.0,
               viewmat=sg.identity_viewmat())
    counts, ids = oracle_lib.tile_lists(params, cam, tile=32)
    assert list(ids) == [2, 0, 1]


@pytest.mark.parametrize("name,sc", SCENES, ids=[n for n, _ in SCENES])
@pytest.mark.parametrize("tile", [16, 8])
def test_work_counts_equal_brute_force(oracle_lib, name, sc, tile):
    p, c = _dicts(sc)
    wc = oracle_lib.work_counts(p, c, tile=tile)
    sp = brute.splats(p, c)
    pairs, evals, tile_evals, contribs = _brute_work(sp, c["width"], c["height"], tile)
    assert wc["pairs"] == pairs
    assert wc["evals"] == evals
    assert wc["tile_evals"] == tile_evals
    assert wc["contribs"] == contribs
    # identities with the oracle's own outputs
    counts, _ = oracle_lib.tile_lists(p, c, tile=tile)
    assert wc["pairs"] == int(counts.sum())
    assert wc["contribs"] == int(oracle_lib.render(p, c)["n"].sum())
    assert wc["tile_evals"] >= wc["evals"] >= wc["contribs"]


def test_work_counts_saturating_scene_stops_early(oracle_lib):
    # on the dense scene most pixels stop: the evaluations are well below
    # what the full lists would cost, and the lockstep count sits between
    name, sc = SCENES[3]
    p, c = _dicts(sc)
    wc = oracle_lib.work_counts(p, c, tile=16)
    r = oracle_lib.render(p, c)
    assert (r["T"] < 1e-3).mean() > 0.5
    counts, _ = oracle_lib.tile_lists(p, c, tile=16)
    full = int(counts.sum()) * 256
    assert wc["tile_evals"] < full
