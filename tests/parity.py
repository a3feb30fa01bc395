"""Element-by-element comparison of the HIP path's outputs with the oracle's.

Bar (fixed by the fixed-point and counter-based design):
  - exact: per-shower counts and energy ledgers; the set of hits and of tree
    nodes of every shower, keyed by path id; their layers, generations,
    parents (compared by the parent's path id) and float energies (both sides
    round E_int * 2^-s once to float32);
  - |d| <= 1e-5 * max(r, 1) for hit coordinates and node vertices, r the
    reference point's distance from the beam axis (the error of a point's
    lateral position scales with how far it has been carried sideways);
  - images: exact integer cell sums, except cells next to a hit lying within
    the coordinate tolerance of a cell edge, which may move one cell.

Near grazing flight (direction almost parallel to the planes) a point's
position is ill-conditioned in the direction: an angle error d(theta) moves
it by (1 + tan^2 theta) d(theta) per unit depth, so single-precision angles
cannot reach the bar there.  Tests of such stress geometries pass
`max_slope` to compare coordinates only where r/z <= max_slope; counts,
keys, energies and layers stay exact everywhere.
"""
from __future__ import annotations

import numpy as np

COORD_RTOL = 1e-5

# The largest coordinate errors met by the checks below in this process
# (outside grazing geometries): relative to max(|component|, 1) -- the bar of
# the scope table, 1e-5 -- and relative to max(r, 1), the bar asserted per
# point (see the module docstring).
COORD_STATS = {"points": 0, "max_rel_component": 0.0, "max_rel_r": 0.0}


def _note_coords(got, ref, r):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    if got.size == 0:
        return
    d = np.abs(got - ref)
    COORD_STATS["points"] += int(got.size)
    COORD_STATS["max_rel_component"] = max(COORD_STATS["max_rel_component"],
                                            float((d / np.maximum(np.abs(ref), 1.0)).max()))
    COORD_STATS["max_rel_r"] = max(COORD_STATS["max_rel_r"], float((d / np.maximum(r, 1.0)).max()))


def to_numpy(out: dict) -> dict:
    r = {}
    for k, v in out.items():
        if hasattr(v, "detach"):
            r[k] = v.detach().cpu().numpy()
        else:
            r[k] = v
    return r


def _f32_energy(e_int, frac_bits):
    return (np.asarray(e_int, np.uint32).astype(np.float32) * np.float32(2.0 ** -frac_bits))


def _coord_ok(got, ref, scale):
    ref = np.asarray(ref, np.float64)
    return np.abs(np.asarray(got, np.float64) - ref) <= COORD_RTOL * np.maximum(scale, 1.0)


def check_counts(gpu: dict, ref: dict, rows=None):
    """counts and ledger of the showers `rows` of the GPU batch (default all)."""
    gc = gpu["counts"] if rows is None else gpu["counts"][rows]
    gl = gpu["ledger"] if rows is None else gpu["ledger"][rows]
    np.testing.assert_array_equal(gc, ref["counts"], err_msg="counts differ")
    np.testing.assert_array_equal(gl.astype(np.uint64), ref["ledger"], err_msg="ledger differs")


def check_hits(gpu: dict, ref: dict, rows=None, geom=None, max_slope=None):
    fb = ref["frac_bits"]
    n = ref["n"]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    base = ref["shower_id_base"]
    order = np.argsort(ref["hit_sid"], kind="stable")
    rs = ref["hit_sid"][order]
    starts = np.searchsorted(rs, base + np.arange(n))
    ends = np.searchsorted(rs, base + np.arange(n), side="right")
    key = gpu["hit_key"].astype(np.uint64)
    for s in range(n):
        g = rows[s]
        off, cnt = int(gpu["hit_offsets"][g]), int(gpu["counts"][g, 1])
        sl = slice(off, off + cnt)
        ri = order[starts[s]:ends[s]]
        assert cnt == len(ri), f"shower {s}: {cnt} hits vs {len(ri)}"
        gk = key[sl]
        go = np.argsort(gk)
        ro = ri[np.argsort(ref["hit_key"][ri])]
        np.testing.assert_array_equal(gk[go], ref["hit_key"][ro], err_msg=f"shower {s}: hit keys")
        np.testing.assert_array_equal(gpu["hit_layer"][sl][go], ref["hit_layer"][ro])
        np.testing.assert_array_equal(gpu["hit_e"][sl][go], _f32_energy(ref["hit_e"][ro], fb),
                                      err_msg=f"shower {s}: hit energies")
        r = np.hypot(ref["hit_x"][ro], ref["hit_y"][ro])
        for c in ("x", "y"):
            if max_slope is None:
                _note_coords(gpu["hit_" + c][sl][go], ref["hit_" + c][ro], r)
            ok = _coord_ok(gpu["hit_" + c][sl][go], ref["hit_" + c][ro], r)
            if max_slope is not None:
                z = geom["z_first"] + ref["hit_plane"][ro] * geom["dz"]
                ok |= r / z > max_slope
            if not ok.all():
                bad = np.nonzero(~ok)[0][0]
                raise AssertionError(f"shower {s}: hit {c} {gpu['hit_' + c][sl][go][bad]} vs "
                                     f"{ref['hit_' + c][ro][bad]}")


def check_tree(gpu: dict, ref: dict, rows=None, max_slope=None):
    fb = ref["frac_bits"]
    n = ref["n"]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    base = ref["shower_id_base"]
    rstart = np.concatenate([[0], np.cumsum(ref["counts"][:, 0])])
    assert np.all(ref["node_sid"] == np.repeat(base + np.arange(n), ref["counts"][:, 0]))
    key = gpu["node_key"].astype(np.uint64)
    for s in range(n):
        g = rows[s]
        off, cnt = int(gpu["node_offsets"][g]), int(gpu["counts"][g, 0])
        sl = slice(off, off + cnt)
        rsl = slice(rstart[s], rstart[s + 1])
        gk, rk = key[sl], ref["node_key"][rsl]
        go, ro = np.argsort(gk), np.argsort(rk)
        np.testing.assert_array_equal(gk[go], rk[ro], err_msg=f"shower {s}: node keys")
        gpar, rpar = gpu["node_parent"][sl], ref["node_parent"][rsl]
        gpk = np.where(gpar >= 0, gk[np.maximum(gpar, 0)], 0)
        rpk = np.where(rpar >= 0, rk[np.maximum(rpar, 0)], 0)
        np.testing.assert_array_equal(gpk[go], rpk[ro], err_msg=f"shower {s}: parents")
        np.testing.assert_array_equal(gpu["node_gen"][sl][go], ref["node_gen"][rsl][ro])
        np.testing.assert_array_equal(gpu["node_e"][sl][go], _f32_energy(ref["node_e"][rsl][ro], fb))
        r = np.hypot(ref["node_vx"][rsl][ro], ref["node_vy"][rsl][ro])
        vz = np.abs(ref["node_vz"][rsl][ro])
        skip = (r / np.maximum(vz, 1e-300) > max_slope) if max_slope is not None else False
        for c, sc in (("vx", r), ("vy", r), ("vz", vz)):
            if max_slope is None and c != "vz":
                _note_coords(gpu["node_" + c][sl][go], ref["node_" + c][rsl][ro], r)
            ok = _coord_ok(gpu["node_" + c][sl][go], ref["node_" + c][rsl][ro], sc) | skip
            assert ok.all(), f"shower {s}: node {c}"


def check_images(gpu: dict, ref: dict, geom: dict, rows=None):
    from oracle import supa_oracle
    n = ref["n"]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    L = gpu["images"].shape[1]
    nx, ny = int(geom["img_nx"]), int(geom["img_ny"])
    x0, x1, y0, y1 = geom["img_x0"], geom["img_x1"], geom["img_y0"], geom["img_y1"]
    ref_img = supa_oracle.images(ref, L, nx, ny, x0, x1, y0, y1)
    want = ref_img.astype(np.float64).astype(np.float32) * np.float32(2.0 ** -ref["frac_bits"])
    got = gpu["images"][rows]
    # hits within the coordinate tolerance of a cell edge may land in a neighbour
    sx, sy = nx / (x1 - x0), ny / (y1 - y0)
    fx = (ref["hit_x"] - x0) * sx
    fy = (ref["hit_y"] - y0) * sy
    rr = np.maximum(np.hypot(ref["hit_x"], ref["hit_y"]), 1.0)
    tx = COORD_RTOL * rr * sx * 2
    ty = COORD_RTOL * rr * sy * 2
    near = (np.abs(fx - np.rint(fx)) <= tx) | (np.abs(fy - np.rint(fy)) <= ty)
    mask = np.zeros(got.shape, bool)
    for h in np.nonzero(near & (ref["hit_layer"] >= 0))[0]:
        s = ref["hit_sid"][h] - ref["shower_id_base"]
        cx, cy = int(np.floor(fx[h])), int(np.floor(fy[h]))
        mask[s, ref["hit_layer"][h], max(cy - 1, 0):cy + 2, max(cx - 1, 0):cx + 2] = True
    diff = got != want
    assert not (diff & ~mask).any(), f"{int((diff & ~mask).sum())} image cells differ"
    return int((diff & mask).sum())


def check_all(gpu: dict, ref: dict, geom: dict, images=False, tree=False, rows=None,
              max_slope=None):
    check_counts(gpu, ref, rows)
    check_hits(gpu, ref, rows, geom, max_slope)
    if tree:
        check_tree(gpu, ref, rows, max_slope)
    if images:
        check_images(gpu, ref, geom, rows)


def tree_path_ids(parent) -> np.ndarray:
    """Path ids of one shower's nodes from their parent indices alone.

    The output layout fixes the numbering: node 0 is the primary (path 1) and
    the two daughters of a split are consecutive, the first of them at an odd
    index, so node 2m+1 has path 2 * path(parent) and node 2m+2 has path
    2 * path(parent) + 1; a parent always precedes its daughters."""
    parent = np.asarray(parent, np.int64)
    n = len(parent)
    path = np.zeros(n, np.uint64)
    if n == 0:
        return path
    assert parent[0] == -1, "node 0 must be the primary"
    j = np.arange(1, n)
    assert ((parent[1:] >= 0) & (parent[1:] < j)).all(), "a parent must precede its daughters"
    assert (parent[2::2] == parent[1:-1:2][:len(parent[2::2])]).all(), \
        "the daughters of a split must be adjacent"
    second = (np.arange(n) % 2 == 0).astype(np.uint64)      # node 2m+2: the second daughter
    known = np.zeros(n, bool)
    path[0], known[0] = 1, True
    par = np.maximum(parent, 0)
    while not known.all():                 # one generation per pass
        todo = ~known & known[par]
        assert todo.any()
        path[todo] = np.uint64(2) * path[par[todo]] + second[todo]
        known[todo] = True
    return path


def with_tree_keys(gpu: dict, rows=None) -> dict:
    """A copy of the GPU outputs with node_key filled in from the tree's
    numbering (outputs written without path ids)."""
    g = dict(gpu)
    key = np.zeros(len(gpu["node_parent"]), np.uint64)
    rows = np.arange(len(gpu["counts"])) if rows is None else np.asarray(rows)
    for i in rows:
        off, cnt = int(gpu["node_offsets"][i]), int(gpu["counts"][i, 0])
        key[off:off + cnt] = tree_path_ids(gpu["node_parent"][off:off + cnt])
    g["node_key"] = key
    return g


def check_hits_unkeyed(gpu: dict, ref: dict, rows=None):
    """Hit clouds written without path ids: per shower, the multiset of
    (layer, energy) is exact, and each hit's coordinates match the oracle's
    hit of the same layer and energy (hits tied on both are matched in x
    order) within the coordinate bar."""
    fb = ref["frac_bits"]
    n = ref["n"]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    base = ref["shower_id_base"]
    order = np.argsort(ref["hit_sid"], kind="stable")
    rs = ref["hit_sid"][order]
    starts = np.searchsorted(rs, base + np.arange(n))
    ends = np.searchsorted(rs, base + np.arange(n), side="right")
    for s in range(n):
        g = rows[s]
        off, cnt = int(gpu["hit_offsets"][g]), int(gpu["counts"][g, 1])
        sl = slice(off, off + cnt)
        ri = order[starts[s]:ends[s]]
        assert cnt == len(ri), f"shower {s}: {cnt} hits vs {len(ri)}"
        # grouped by plane: layers never decrease along a segment when the
        # layer map is monotone (identity here)
        ge = np.asarray(gpu["hit_e"][sl], np.float32)
        re = _f32_energy(ref["hit_e"][ri], fb)
        gk = np.lexsort((np.asarray(gpu["hit_x"][sl], np.float64), ge, gpu["hit_layer"][sl]))
        rk = np.lexsort((ref["hit_x"][ri], re, ref["hit_layer"][ri]))
        np.testing.assert_array_equal(gpu["hit_layer"][sl][gk], ref["hit_layer"][ri][rk],
                                      err_msg=f"shower {s}: layers")
        np.testing.assert_array_equal(ge[gk], re[rk], err_msg=f"shower {s}: hit energies")
        r = np.hypot(ref["hit_x"][ri][rk], ref["hit_y"][ri][rk])
        for c in ("x", "y"):
            ok = _coord_ok(gpu["hit_" + c][sl][gk], ref["hit_" + c][ri][rk], r)
            if not ok.all():
                bad = np.nonzero(~ok)[0][0]
                raise AssertionError(f"shower {s}: hit {c} {gpu['hit_' + c][sl][gk][bad]} vs "
                                     f"{ref['hit_' + c][ri][rk][bad]}")


def check_same_outputs(a, b, images=True):
    """Two runs of one call through different entry points or launch
    settings: equal bit for bit (the order of records within a plane and the
    numbering of nodes may differ, so hits and nodes are compared in path-id
    order and parents by their path ids)."""
    a, b = to_numpy(a), to_numpy(b)
    assert a["total_hits"] == b["total_hits"] and a["total_nodes"] == b["total_nodes"]
    assert a["total_steps"] == b["total_steps"]
    for k in ("counts", "ledger", "hit_offsets", "node_offsets") + (("images",) if images else ()):
        if k in a or k in b:
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    n = a["counts"].shape[0]
    for pre, off, col, fields in (("hit", "hit_offsets", 1, ("x", "y", "e", "layer", "key")),
                                  ("node", "node_offsets", 0, ("gen", "vx", "vy", "vz", "e", "key"))):
        if off not in a:
            continue
        for i in range(n):
            sl = slice(int(a[off][i]), int(a[off][i]) + int(a["counts"][i, col]))
            ka, kb = a[pre + "_key"][sl], b[pre + "_key"][sl]
            oa, ob = np.argsort(ka), np.argsort(kb)
            for f in fields:
                np.testing.assert_array_equal(a[f"{pre}_{f}"][sl][oa], b[f"{pre}_{f}"][sl][ob],
                                              err_msg=f"shower {i}: {pre}_{f}")
            if pre == "node":
                pa, pb = a["node_parent"][sl], b["node_parent"][sl]
                pka = np.where(pa >= 0, ka[np.maximum(pa, 0)], 0)
                pkb = np.where(pb >= 0, kb[np.maximum(pb, 0)], 0)
                np.testing.assert_array_equal(pka[oa], pkb[ob], err_msg=f"shower {i}: parents")


def check_valid_shower(gpu: dict, i: int):
    """A shower that cannot be compared with the oracle (a choice taken on
    float coordinates within rounding of a boundary) must still be a valid
    outcome of the process: exact ledger (E0 = stopped + cut + escaped),
    nodes = 1 + 2 splits, hits + escaped = splits + 1, each split's two
    daughters adjacent and carrying their parent's energy between them, and
    path ids unique among the shower's hits and nodes."""
    led = gpu["ledger"][i].astype(np.uint64)
    cnt = gpu["counts"][i]
    assert led[1] + led[2] + led[3] == led[0], "ledger"
    assert cnt[0] == 1 + 2 * cnt[3], "nodes vs splits"
    assert cnt[1] + cnt[4] == cnt[3] + 1, "hits + escaped vs splits"
    no, nn = int(gpu["node_offsets"][i]), int(cnt[0])
    par = gpu["node_parent"][no:no + nn]
    keys = tree_path_ids(par)
    if "node_key" in gpu:
        np.testing.assert_array_equal(gpu["node_key"][no:no + nn].astype(np.uint64), keys)
    e = gpu["node_e"][no:no + nn].astype(np.float64)
    for a in range(1, nn, 2):
        # float energies: each rounded once from the exact integer split
        assert abs(e[a] + e[a + 1] - e[par[a]]) <= 2 * np.spacing(np.float32(max(e[par[a]], 1e-30))), a
    ho, nh = int(gpu["hit_offsets"][i]), int(cnt[1])
    if "hit_key" in gpu:
        hk = gpu["hit_key"][ho:ho + nh].astype(np.uint64)
        assert len(np.unique(hk)) == nh, "hit path ids repeat"
