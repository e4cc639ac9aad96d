"""Pins of the oracle's discrete structure (CPU only).

App. A.1.1: crossing edges of a cell are grouped into at most four
partitions (the primal polygons of the 22 Dual-Marching-Cubes
configurations), and the manifold fix makes the output manifold.
"""
import itertools

import numpy as np
import pytest

import odc_inputs as I
import meshcheck as M

# cube-local corner c = x + 2y + 4z; cell-local edge 4*axis + o1 + 2*o2


def _edge_corners(le):
    axis = le // 4
    others = [a for a in range(3) if a != axis]
    off = [0, 0, 0]
    off[others[0]] = le & 1
    off[others[1]] = (le >> 1) & 1
    c0 = off[0] + 2 * off[1] + 4 * off[2]
    off[axis] = 1
    c1 = off[0] + 2 * off[1] + 4 * off[2]
    return c0, c1


def _sym_group():
    """All 48 rigid and mirror maps of the cube, as corner permutations and
    edge permutations."""
    out = []
    for perm in itertools.permutations(range(3)):
        for flips in itertools.product((0, 1), repeat=3):
            def cmap(c, perm=perm, flips=flips):
                b = [(c >> a) & 1 for a in range(3)]
                nb = [0, 0, 0]
                for a in range(3):
                    nb[perm[a]] = b[a] ^ flips[perm[a]]
                return nb[0] + 2 * nb[1] + 4 * nb[2]
            cp = [cmap(c) for c in range(8)]
            ep = []
            for le in range(12):
                a, b = _edge_corners(le)
                na, nb_ = sorted((cp[a], cp[b]))
                ep.append(next(x for x in range(12) if sorted(_edge_corners(x)) == [na, nb_]))
            out.append((cp, ep))
    return out


def _crossing(cfg):
    return [le for le in range(12)
            if ((cfg >> _edge_corners(le)[0]) & 1) != ((cfg >> _edge_corners(le)[1]) & 1)]


def _partition_sets(O, cfg, flipmask=0):
    n, pm = O.cube_partitions(cfg, flipmask)
    parts = {}
    for le in _crossing(cfg):
        parts.setdefault((pm >> (2 * le)) & 3, set()).add(le)
    assert len(parts) == n
    return n, {frozenset(s) for s in parts.values()}


def test_configuration_classes_burnside():
    """256 configurations fall into 22 classes under rotation and mirroring
    (App. A.1.1, Fig. A1)."""
    G = _sym_group()
    assert len(G) == 48
    seen, classes = set(), 0
    for cfg in range(256):
        if cfg in seen:
            continue
        classes += 1
        for cp, _ in G:
            seen.add(sum(((cfg >> c) & 1) << cp[c] for c in range(8)))
    assert classes == 22


def test_partitions_histogram_and_max_four(oracle_mod):
    hist = {}
    four = []
    for cfg in range(256):
        n, _ = _partition_sets(oracle_mod, cfg)
        hist[n] = hist.get(n, 0) + 1
        if n == 4:
            four.append(cfg)
    assert max(hist) == 4
    assert hist == {0: 2, 1: 162, 2: 82, 3: 8, 4: 2}
    assert four == [105, 150]


def test_partitions_equivariant_under_48_symmetries(oracle_mod):
    G = _sym_group()
    for cfg in range(256):
        n, parts = _partition_sets(oracle_mod, cfg)
        for cp, ep in G:
            cfg2 = sum(((cfg >> c) & 1) << cp[c] for c in range(8))
            _, parts2 = _partition_sets(oracle_mod, cfg2)
            mapped = {frozenset(ep[e] for e in s) for s in parts}
            assert mapped == parts2, (cfg, cp)


def _components(nodes, adj):
    nodes = set(nodes)
    comp = 0
    while nodes:
        stack = [nodes.pop()]
        comp += 1
        while stack:
            x = stack.pop()
            for y in adj.get(x, ()):
                if y in nodes:
                    nodes.remove(y)
                    stack.append(y)
    return comp


def test_partition_count_by_surface_regions(oracle_mod):
    """Independent count: on the cube surface (a sphere) k disjoint curves
    cut k+1 regions, so #partitions = #inside regions + #outside regions - 1.
    Pairing around inside corners keeps inside corners apart on a
    checkerboard face, so outside corners connect across its diagonal; the
    flipped pairing does the opposite on that face."""
    faces = []
    for a in range(3):
        u, v = [x for x in range(3) if x != a]
        for s in (0, 1):
            cs = []
            for lc in range(4):
                off = [0, 0, 0]
                off[a], off[u], off[v] = s, lc & 1, lc >> 1
                cs.append(off[0] + 2 * off[1] + 4 * off[2])
            faces.append(cs)
    rng = np.random.default_rng(0)
    for cfg in range(1, 255):
        for flipmask in [0] + list(rng.integers(0, 64, 3)):
            lab = [(cfg >> c) & 1 for c in range(8)]
            adj = {}
            for le in range(12):
                c0, c1 = _edge_corners(le)
                if lab[c0] == lab[c1]:
                    adj.setdefault(c0, []).append(c1)
                    adj.setdefault(c1, []).append(c0)
            for lf, cs in enumerate(faces):
                L = [lab[c] for c in cs]
                if L[0] == L[3] != L[1] == L[2]:
                    inside_pair = (cs[0], cs[3]) if L[0] == 1 else (cs[1], cs[2])
                    outside_pair = (cs[1], cs[2]) if L[0] == 1 else (cs[0], cs[3])
                    link = inside_pair if (flipmask >> lf) & 1 else outside_pair
                    adj.setdefault(link[0], []).append(link[1])
                    adj.setdefault(link[1], []).append(link[0])
            nin = _components([c for c in range(8) if lab[c]], adj)
            nout = _components([c for c in range(8) if not lab[c]], adj)
            n, _ = oracle_mod.cube_partitions(cfg, int(flipmask))
            assert n == nin + nout - 1, (cfg, flipmask)


def test_complement_swaps_pairing_rule(oracle_mod):
    """Complementing the labels turns 'around inside corners' into 'around
    outside corners': partitions(~cfg, all flipped) == partitions(cfg)."""
    for cfg in range(256):
        _, a = _partition_sets(oracle_mod, cfg, 0)
        _, b = _partition_sets(oracle_mod, 255 - cfg, 63)
        assert a == b


def _labels_field(labels, N):
    """CSG field whose corner labels equal `labels` ((N+1)^3 bools, x fastest):
    a small sphere around every inside corner."""
    h = 1.0 / N
    recs = []
    idx = np.argwhere(labels.reshape(N + 1, N + 1, N + 1))
    for k, j, i in idx:
        recs.append(I.sphere_record((-0.5 + i * h, -0.5 + j * h, -0.5 + k * h), 0.3 * h))
    if not recs:
        recs.append(I.sphere_record((5.0, 5.0, 5.0), 0.1))
    return I.csg_field(recs)


@pytest.mark.parametrize("seed", range(4))
def test_random_labels_give_closed_manifold(oracle_mod, seed):
    """Brute force of the manifold guarantee (App. A.1.1): random corner labels
    in the interior of a 7^3 grid, bordered by outside corners, many ambiguous
    faces; the mesh is a closed oriented 2-manifold."""
    N = 7
    rng = np.random.default_rng(seed)
    lab = np.zeros((N + 1, N + 1, N + 1), bool)
    lab[1:N, 1:N, 1:N] = rng.uniform(size=(N - 1, N - 1, N - 1)) < 0.45
    f = _labels_field(lab, N)
    g = I.unit_grid(N, 8)
    m = oracle_mod.Oracle(f, g).mesh()
    assert np.array_equal(m["corner_label"].astype(bool), lab.reshape(-1))
    ok, why = M.is_closed_oriented_manifold(m["tris"], len(m["vert"]))
    assert ok, why
    # vertex / triangle identities of the emission (App. A.1.5)
    quads = int(np.sum(m["edge_case"] > 0))
    assert len(m["tris"]) == 2 * quads + 2 * m["n_case3"]
    assert len(m["vert"]) == int(m["cell_npart"].sum()) + m["n_case3"]


def test_manifold_fix_two_cell_blocks(oracle_mod):
    """All 2^12 label configurations of two x-adjacent cells: after the flip no
    shared ambiguous face has both pairs merged in both cells."""
    bad_before = bad_after = 0
    for code in range(1 << 12):
        # corners of cell A (x=0..1) and cell B (x=1..2): 12 corners (x,y,z)
        lab = {}
        for n in range(12):
            x, y, z = n % 3, (n // 3) % 2, n // 6
            lab[(x, y, z)] = (code >> n) & 1
        cfgA = sum(lab[(c & 1, (c >> 1) & 1, c >> 2)] << c for c in range(8))
        cfgB = sum(lab[(1 + (c & 1), (c >> 1) & 1, c >> 2)] << c for c in range(8))
        # shared face: x side 1 of A (local face 1), x side 0 of B (local face 0)
        L = [lab[(1, 0, 0)], lab[(1, 1, 0)], lab[(1, 0, 1)], lab[(1, 1, 1)]]
        if not (L[0] == L[3] != L[1] == L[2]):
            continue

        def merged(cfg, lf, flip):
            n, pm = oracle_mod.cube_partitions(cfg, flip << lf)
            # face-local edges 0 and 1 lie in different pairs on every
            # checkerboard face; map them to cell-local edges (normal x:
            # u = y, v = z) -> y-edges with x offset = side
            side = lf & 1
            e0 = 4 * 1 + side + 2 * 0   # y-edge at (x=side, z=0)
            e1 = 4 * 1 + side + 2 * 1   # y-edge at (x=side, z=1)
            return ((pm >> (2 * e0)) & 3) == ((pm >> (2 * e1)) & 3)

        b = merged(cfgA, 1, 0) and merged(cfgB, 0, 0)
        bad_before += b
        flip = 1 if b else 0
        bad_after += merged(cfgA, 1, flip) and merged(cfgB, 0, flip)
    assert bad_before == 18  # of the 512 blocks whose shared face is ambiguous
    assert bad_after == 0
