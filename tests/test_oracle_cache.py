"""Pins of the oracle's residency-aware LOD cut (Sec 5.2 request queue and
fallback to the parent block, Sec 4.2 GPU cache), on the CPU.

Checked against the cut with every node resident, against brute-force
enumeration of the definition on tiny trees, and against the partition
property of a cut."""
import numpy as np
import pytest

import gen
import oracle as O

O.build()


def all_nodes(dims0, B, levels):
    out = []
    for L in range(levels):
        g = O.brick_grid(dims0, B, L)
        for z in range(g[2]):
            for y in range(g[1]):
                for x in range(g[0]):
                    out.append((L, x, y, z))
    return out


def ident(n):
    return O.node_id(*n)


def children(dims0, B, n):
    L, x, y, z = n
    if L == 0:
        return []
    g = O.brick_grid(dims0, B, L - 1)
    return [(L - 1, 2 * x + dx, 2 * y + dy, 2 * z + dz)
            for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)
            if 2 * x + dx < g[0] and 2 * y + dy < g[1] and 2 * z + dz < g[2]]


def brute(dims0, B, levels, view, resident, tau, bias, lod):
    """The definition, node by node: n is in the cut iff every ancestor a
    does not suit and has all its children resident, and n itself suits or
    has a missing child. Requests: the missing children of cut nodes that do
    not suit, save those outside every ray of the view."""
    e = np.asarray(view["cam_to_world"], dtype=np.float64).reshape(4, 4)[:3, 3]
    K = O.lod_k(view, tau)
    res = set(int(r) for r in resident)

    def suits(n):
        if not lod:
            return n[0] == bias
        return O.node_accept(dims0, B, e, K, bias, n[0], n[1:])

    def descends(a):
        return (not suits(a)) and all(ident(c) in res for c in children(dims0, B, a))

    cut, req = [], []
    for n in all_nodes(dims0, B, levels):
        L = n[0]
        if L < bias:
            continue
        ok = True
        a = n
        for l in range(L + 1, levels):
            a = (l, n[1] >> (l - L), n[2] >> (l - L), n[3] >> (l - L))
            if not descends(a):
                ok = False
                break
        if not ok or descends(n):
            continue
        cut.append(ident(n))
        if not suits(n):
            req += [ident(c) for c in children(dims0, B, n)
                    if ident(c) not in res
                    and not O.box_outside_view(view, *O.node_box(dims0, B, c[0], c[1:]))]
    return np.array(sorted(cut), np.uint64), np.array(sorted(req), np.uint64)


def tiny_views(rng, dims0, k):
    c = np.asarray(dims0, float) / 2
    out = []
    for _ in range(k):
        eye = c + rng.normal(size=3) * rng.uniform(0.2, 3.0) * np.linalg.norm(dims0)
        out.append(gen.view(gen.look_at(eye, c + rng.normal(size=3)), 17, 13,
                            rng.uniform(0.2, 1.0)))
    return out


def test_every_node_resident_gives_the_plain_cut():
    dims0, B, levels = (64, 48, 40), 4, 4
    ids = [ident(n) for n in all_nodes(dims0, B, levels)]
    rng = np.random.default_rng(80)
    for v in tiny_views(rng, dims0, 20):
        for bias in (0, 1):
            cut, req = O.lod_cut_resident(dims0, B, levels, v, ids, tau=1.0, bias=bias)
            assert np.array_equal(cut, O.lod_cut(dims0, B, levels, v, 1.0, bias))
            assert len(req) == 0


@pytest.mark.parametrize("dims0,B,levels", [((16, 16, 16), 2, 4), ((13, 9, 11), 2, 4),
                                            ((40, 24, 32), 4, 3)])
def test_residency_cut_equals_brute_force_definition(dims0, B, levels):
    rng = np.random.default_rng(81)
    nodes = all_nodes(dims0, B, levels)
    top = [n for n in nodes if n[0] == levels - 1]
    for trial in range(40):
        p = rng.uniform(0.3, 1.0)
        res = [ident(n) for n in nodes if n[0] == levels - 1 or rng.uniform() < p]
        v = tiny_views(rng, dims0, 1)[0]
        tau = rng.choice([0.5, 1.0, 4.0])
        bias = int(rng.integers(0, levels))
        lod = bool(rng.uniform() < 0.8)
        cut, req = O.lod_cut_resident(dims0, B, levels, v, res, tau=tau, bias=bias, lod=lod)
        bc, br = brute(dims0, B, levels, v, res, tau, bias, lod)
        assert np.array_equal(cut, bc), trial
        assert np.array_equal(req, br), trial
        # the cut is resident and covers every level-0 cell exactly once
        assert set(cut.tolist()) <= set(res)
        cover = np.zeros(O.brick_grid(dims0, B, 0)[::-1], np.int32)
        for L, x, y, z in O.node_decode(cut):
            s = 1 << L
            cover[z * s:(z + 1) * s, y * s:(y + 1) * s, x * s:(x + 1) * s] += 1
        assert np.all(cover == 1)
    assert len(top) >= 1


def test_missing_top_level_node_is_an_error():
    dims0, B, levels = (16, 16, 16), 4, 2
    v = gen.view(gen.look_at((-20, 30, 25), (8, 8, 8)), 9, 7, 0.5)
    with pytest.raises(ValueError):
        O.lod_cut_resident(dims0, B, levels, v, [O.node_id(0, 0, 0, 0)])


def test_nothing_below_the_top_gives_the_top_level_and_requests_its_children():
    dims0, B, levels = (32, 32, 32), 4, 3
    v = gen.view(gen.look_at((-5, 40, 30), (16, 16, 16)), 33, 21, 0.9)
    top = [ident(n) for n in all_nodes(dims0, B, levels) if n[0] == 2]
    cut, req = O.lod_cut_resident(dims0, B, levels, v, top)
    assert np.array_equal(cut, np.array(sorted(top), np.uint64))
    full = O.lod_cut(dims0, B, levels, v)
    wanted_children = set()
    for L, x, y, z in O.node_decode(full):
        if L < 2:
            a = (1, x >> (1 - L), y >> (1 - L), z >> (1 - L))
            if not O.box_outside_view(v, *O.node_box(dims0, B, 1, a[1:])):
                wanted_children.add(ident(a))
    assert len(wanted_children) > 0
    assert set(req.tolist()) >= wanted_children
    assert all(int(r) >> 60 == 1 for r in req)


def test_culling_keeps_every_box_a_pixel_ray_enters():
    """Sec 5.2 leaves out blocks no ray sees. Pinned against the rays
    themselves: every node box that the ray of some pixel enters (at a
    positive parameter) is kept, and boxes behind the eye or beside the
    image are culled."""
    rng = np.random.default_rng(83)
    dims0, B, levels = (48, 40, 32), 4, 3
    boxes = [(n, O.node_box(dims0, B, n[0], n[1:])) for n in all_nodes(dims0, B, levels)]
    culled_any = 0
    for v in tiny_views(rng, dims0, 12):
        hit = set()
        for py in range(v["height"]):
            for px in range(v["width"]):
                e, d = O.ray(v, px, py)
                for n, (lo, hi) in boxes:
                    ok, t0, t1 = O.box_interval(e, d, lo, hi)
                    if ok and t1 > 0.0:
                        hit.add(n)
        for n, (lo, hi) in boxes:
            out = O.box_outside_view(v, lo, hi)
            assert not (out and n in hit), (n, v["cam_to_world"])
            culled_any += out
    assert culled_any > 0
    # a box behind the eye is culled; a lens view culls nothing
    v = gen.view(gen.look_at((0, 0, 0), (0, 0, -10)), 9, 7, 0.5)
    assert O.box_outside_view(v, (-1, -1, 5), (1, 1, 6))
    assert not O.box_outside_view(v, (-1, -1, -6), (1, 1, -5))
    lens = dict(v, lens=[0.2, 0.1, 0.0, 0.0])
    assert not O.box_outside_view(lens, (-1, -1, 5), (1, 1, 6))
