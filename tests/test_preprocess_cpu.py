"""The library's host preprocessing against the oracle (no device work, so
these run without a GPU).

* chordal extension and maximal cliques (sdp_pattern_*): bit-exact -- the
  same extended pattern, the same cliques in the same order -- on grids,
  cycles, random graphs and the 45 x 45 grid of the nonchordal workload;
  the index map and the instance remapping;
* data scaling (sdp_scale_*): factors, scaled data and recovered solutions
  within 1e-12 relative (the two sum in different orders); dense and CSR A.
"""
import numpy as np
import pytest

import sdpgen
from cases import as_instance
from oracle import preprocess as pp


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def pattern_cases():
    out = [("cycle9", 9, *sdpgen.cycle_pattern(9)), ("grid7x5", 35, *sdpgen.grid_pattern(7, 5)),
           ("grid45", 2025, *sdpgen.grid_pattern(45, 45))]
    for seed in range(4):
        out.append((f"rand{seed}", 120, *sdpgen.random_sparse_pattern(120, 3.0, seed)))
    out.append(("isolated", 5, np.arange(5, dtype=np.int32), np.arange(5, dtype=np.int32)))
    return out


@pytest.mark.parametrize("name,n,pr,pc", pattern_cases())
def test_extension_matches_oracle(sdp, name, n, pr, pc):
    P = sdp.chordal_extension(n, pr, pc)
    er, ec, cl = pp.chordal_extension(n, pr, pc)
    assert np.array_equal(P.pat_row, er) and np.array_equal(P.pat_col, ec)
    assert [c.tolist() for c in P.cliques()] == cl


def test_input_in_either_triangle_with_duplicates(sdp):
    pr, pc = sdpgen.grid_pattern(4, 4)
    ref = sdp.chordal_extension(16, pr, pc)
    # upper-triangle copies, duplicates and a shuffled order give the same result
    rng = np.random.default_rng(1)
    r2 = np.concatenate([pc, pr, pr])
    c2 = np.concatenate([pr, pc, pc])
    perm = rng.permutation(r2.shape[0])
    P = sdp.chordal_extension(16, r2[perm], c2[perm])
    assert np.array_equal(P.pat_row, ref.pat_row) and np.array_equal(P.pat_col, ref.pat_col)
    assert np.array_equal(P.clique_vert, ref.clique_vert)


def test_index_map(sdp):
    pr, pc = sdpgen.grid_pattern(5, 6)
    P = sdp.chordal_extension(30, pr, pc)
    idx = P.index_of(pr, pc)
    assert (idx >= 0).all()
    assert np.array_equal(P.pat_row[idx], pr) and np.array_equal(P.pat_col[idx], pc)
    assert np.array_equal(P.index_of(pc, pr), idx)               # upper triangle
    # a pair the extension does not hold maps to -1
    full = {(int(r), int(c)) for r, c in zip(P.pat_row, P.pat_col)}
    miss = next((r, c) for r in range(30) for c in range(r) if (r, c) not in full)
    assert P.index_of([miss[0]], [miss[1]])[0] == -1


def test_pattern_errors(sdp):
    with pytest.raises(sdp.SdpError) as e:
        sdp.chordal_extension(0, [], [])
    assert e.value.code == -1
    with pytest.raises(sdp.SdpError) as e:
        sdp.chordal_extension(4, [4], [0])
    assert e.value.code == -1
    with pytest.raises(sdp.SdpError):
        sdp.chordal_extension(4, [1], [-1])


@pytest.mark.parametrize("density", [None, 0.3])
def test_extend_instance(sdp, oracle_mod, density):
    from cases import oracle_extended
    pr, pc = sdpgen.grid_pattern(4, 5)
    inst = sdpgen.instance_on_pattern(20, pr, pc, 7, seed=2, density=density)
    ext = sdp.extend_instance(inst)
    ref = oracle_extended(inst)
    assert np.array_equal(ext.pat_row, ref.pat_row) and np.array_equal(ext.clique_vert, ref.clique_vert)
    assert np.array_equal(ext.clique_ptr, ref.clique_ptr)
    assert np.array_equal(as_instance(ext).a_dense(), ref.a_val)
    assert np.array_equal(ext.c, ref.c) and np.array_equal(ext.b, ref.b)
    # the oracle accepts it as a valid decomposed instance
    oracle_mod.Problem(as_instance(ext))


def scaling_cases():
    base = sdpgen.block_arrow_instance(3, 4, 2, 8, seed=1)
    sparse = sdpgen.block_arrow_instance(4, 5, 2, 12, seed=2, density=0.3)
    return [base, sdpgen.rescaled_instance(base, seed=3), sparse,
            sdpgen.rescaled_instance(sparse, seed=4)]


@pytest.mark.parametrize("k", range(4))
@pytest.mark.parametrize("iters", [0, 1, 10])
def test_scaling_matches_oracle(sdp, k, iters):
    inst = scaling_cases()[k]
    S = sdp.scale_instance(inst, iters=iters)
    e, s, rb, sc = pp.equilibrate(inst, iters)
    assert rel(S.row_scale, e) <= 1e-12 and rel(S.vertex_scale, s) <= 1e-12
    assert abs(S.rho_b - rb) <= 1e-12 * rb and abs(S.sigma_c - sc) <= 1e-12 * sc
    a, b, c = pp.scale_data(inst, e, s, rb, sc)
    assert rel(as_instance(S.scaled).a_dense(), a) <= 1e-12
    assert rel(S.scaled.b, b) <= 1e-12 and rel(S.scaled.c, c) <= 1e-12
    rng = np.random.default_rng(k)
    x, y, z = rng.standard_normal(inst.nnz), rng.standard_normal(inst.m), rng.standard_normal(inst.nnz)
    xl, yl, zl = S.recover(x, y, z)
    xo, yo, zo = pp.recover(inst, e, s, rb, sc, x, y, z)
    assert rel(xl, xo) <= 1e-12 and rel(yl, yo) <= 1e-12 and rel(zl, zo) <= 1e-12


def test_scaling_errors(sdp):
    inst = sdpgen.block_arrow_instance(2, 2, 1, 3, seed=0)
    with pytest.raises(sdp.SdpError):
        sdp.scale_instance(inst, iters=-1)
    bad = sdpgen.block_arrow_instance(2, 2, 1, 3, seed=0)
    bad.b = bad.b.copy()
    bad.b[0] = np.inf
    with pytest.raises(sdp.SdpError) as e:
        sdp.scale_instance(bad)
    assert e.value.code == -6
