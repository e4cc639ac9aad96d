"""Pins of the oracle's replay (staged parity) mode, on the CPU.

The paper fixes no precision, so an occupancy decision whose logit lies
within the evaluation error of 0 may go either way.  For a checked run the
implementation records the label of every query it made; the oracle follows
that branch at its own near-ties and counts every other disagreement.  These
tests pin the encoding of those records and the replay semantics to things
other than the replay code: the closed-form relation between a bisection's
decisions and its final bracket (Sec. 5.1), planted disagreements, and the
untraced oracle's own results.
"""
import numpy as np

import odc_inputs as I


def _trace_of(O, m, **kw):
    """A trace holding the oracle run m's own decisions."""
    words = np.packbits(m["corner_label"], bitorder="little")
    words = np.pad(words, (0, (-len(words)) % 4)).view(np.uint32)
    rec = (m["pair_face"].astype(np.int64) * 2 + (m["pair_info"] & 1)).astype(np.int32)
    return O.Trace(label_words=words, edge_ids=m["edge_id"], edge_bits=m["edge_bits"],
                   edge_t=m["edge_t"].astype(np.float32), pair_rec=rec, pair_bits=m["pair_bits"],
                   pair_pf=m["pair_pf"], **kw)


def _lower_label(m, e, N):
    n1 = N + 1
    ea = N * n1 * n1
    a, loc = int(e) // ea, int(e) % ea
    dims = [n1, n1, n1]
    dims[a] = N
    p = [loc % dims[0], (loc // dims[0]) % dims[1], loc // (dims[0] * dims[1])]
    return int(m["corner_label"][p[0] + n1 * (p[1] + n1 * p[2])])


def _bits_from_t(t, label0, k):
    """Sec. 5.1 with the midpoint rule: after k halvings the bracket is
    [lo, lo + 2^-k] and t = lo + 2^-(k+1); halving i kept the lower end's
    label (lo moved up) exactly when bit i of lo's binary fraction is 1."""
    lo = t - 2.0 ** -(k + 1)
    bits = 0
    for i in range(1, k + 1):
        moved_up = int(np.floor(lo * 2 ** i)) & 1
        lab = label0 if moved_up else 1 - label0
        bits |= lab << (i - 1)
    return bits


def test_edge_bits_follow_from_the_bracket(oracle_mod):
    """Every crossing edge's recorded labels are those the final bracket
    implies (closed form), on the sphere (binary32 labels, no near-ties)."""
    f, g = I.sphere_case(12, 10)
    m = oracle_mod.Oracle(f, g).mesh()
    assert len(m["edge_id"]) > 100
    for e, t, b in zip(m["edge_id"], m["edge_t"], m["edge_bits"]):
        assert int(b) == _bits_from_t(t, _lower_label(m, e, g.res), g.iters_1d), int(e)


def test_pair_bits_mark_the_queries_made(oracle_mod):
    """The oracle queries m, all of step 1, and both step-2 rays unless q
    coincides with m (then it stops after step 1)."""
    f, g = I.csg_random_field(2), I.unit_grid(16, 15)
    m = oracle_mod.Oracle(f, g).mesh()
    n1 = 1 + g.lin1 + g.bin1
    full = (1 << (n1 + 2 * (g.lin2 + g.bin2))) - 1
    qm = (m["pair_info"] >> 13) & 1
    ev = m["pair_bits"][:, 1].astype(np.uint64)
    assert np.all(ev[qm == 0] == np.uint64(full))
    assert np.all(ev[qm == 1] == np.uint64((1 << n1) - 1))
    assert np.all((m["pair_bits"][:, 0] & ~m["pair_bits"][:, 1]) == 0)


def test_self_replay_is_the_identity(oracle_mod):
    """Replaying the oracle's own decisions changes nothing, adopts exactly
    its near-ties and clears their flags; staged with its own 1D and 2D
    points it is the same again."""
    f, g = I.mlp_field(3), I.unit_grid(12, 15)
    m0 = oracle_mod.Oracle(f, g, mlp_tie_eps=1e-5).mesh()
    ties = int(m0["corner_tie"].sum()) + int((m0["edge_tie_step"] > 0).sum())
    for staged in (False, True):
        tr = _trace_of(oracle_mod, m0, staged=staged)
        m1 = oracle_mod.Oracle(f, g, mlp_tie_eps=1e-5, trace=tr).mesh()
        assert tr.mismatched == 0 and tr.unmatched == 0
        assert tr.adopted >= ties
        for k in ("corner_label", "edge_id", "edge_t", "edge_bits", "pair_face", "pair_pf",
                  "pair_bits", "cell_id", "cell_partmap", "vert", "tris", "edge_case"):
            assert np.array_equal(m0[k], m1[k]), (staged, k)
        assert not m1["corner_tie"].any() and not (m1["edge_tie_step"] > 0).any()
        assert not m1["pair_tie"].any()


def test_disagreement_away_from_a_tie_is_counted(oracle_mod):
    """A recorded label that differs where the oracle's decision is clear is
    a failure of the implementation: counted, and the oracle keeps its own."""
    f, g = I.sphere_case(10, 10)
    m0 = oracle_mod.Oracle(f, g).mesh()
    bits = m0["edge_bits"].copy()
    bits[7] ^= 1 << 4
    pb = m0["pair_bits"].copy()
    pb[3, 0] ^= np.uint64(1)          # the label of m
    m0b = dict(m0, edge_bits=bits, pair_bits=pb)
    tr = _trace_of(oracle_mod, m0b)
    m1 = oracle_mod.Oracle(f, g, trace=tr).mesh()
    assert tr.mismatched == 2 and tr.adopted == 0
    assert np.array_equal(m1["edge_t"], m0["edge_t"])
    assert np.array_equal(m1["pair_pf"], m0["pair_pf"])


def test_near_ties_follow_the_recorded_branch(oracle_mod):
    """With every MLP decision a near-tie (a band wider than any logit), the
    bisection follows arbitrary recorded labels: the 1D point is the one the
    closed form gives for those decisions, and every 2D-search query takes
    the recorded label."""
    f, g = I.mlp_field(3), I.unit_grid(8, 12)
    m0 = oracle_mod.Oracle(f, g, mlp_tie_eps=1e-5).mesh()
    rng = np.random.default_rng(11)
    ebits = rng.integers(0, 1 << g.iters_1d, len(m0["edge_id"])).astype(np.uint32)
    pbits = rng.integers(0, 2 ** 63, (len(m0["pair_face"]), 2), dtype=np.uint64)
    pbits[:, 1] = np.uint64(2 ** 64 - 1)
    tr = _trace_of(oracle_mod, dict(m0, edge_bits=ebits, pair_bits=pbits))
    m1 = oracle_mod.Oracle(f, g, mlp_tie_eps=1e30, trace=tr).mesh()
    assert tr.mismatched == 0 and tr.unmatched == 0
    k = g.iters_1d
    for x, e in enumerate(m1["edge_id"]):
        l0 = _lower_label(m1, e, g.res)
        lo = 0.0
        for i in range(1, k + 1):
            if ((int(ebits[x]) >> (i - 1)) & 1) == l0:
                lo += 2.0 ** -i
        assert m1["edge_t"][x] == lo + 2.0 ** -(k + 1), x
    made = m1["pair_bits"][:, 1]
    assert np.all((m1["pair_bits"][:, 0] ^ pbits[:, 0]) & made == 0)
    assert np.array_equal(m1["edge_bits"], ebits)


def test_labels_given_topology(oracle_mod):
    """Topology from given labels without evaluating the field equals the
    full pipeline's (the whole-grid check at full resolution uses it)."""
    f, g = I.csg_random_field(2), I.unit_grid(20, 15)
    m0 = oracle_mod.Oracle(f, g).mesh()
    words = np.packbits(m0["corner_label"], bitorder="little")
    words = np.pad(words, (0, (-len(words)) % 4)).view(np.uint32)
    bad = I.csg_field([I.sphere_record((9.0, 9.0, 9.0), 0.1)])  # never evaluated
    tr = oracle_mod.Trace(label_words=words, labels_given=True)
    m1 = oracle_mod.Oracle(bad, g, trace=tr, topology_only=True).mesh()
    for k in ("corner_label", "edge_id", "pair_face", "cell_id", "cell_npart",
              "cell_partmap", "cell_flipmask", "cell_vbase"):
        assert np.array_equal(m0[k], m1[k]), k
    structural = ~(1 << 13)  # all but the search's q == m bit
    assert np.array_equal(m0["pair_info"] & structural, m1["pair_info"] & structural)
    assert m1["n_flipped_faces"] == m0["n_flipped_faces"]
    assert len(m1["tris"]) == 0
