"""Shared test inputs (seeded instances and invalid variants)."""
import copy

import numpy as np

import sdpgen


def invalid_instances():
    """(name, instance, expected status) for the validation paths."""
    base = sdpgen.block_arrow_instance(3, 3, 2, 5, seed=0)
    out = []
    # a pattern coordinate no clique covers (vertex 4 of block 1 with vertex 0 of block 0)
    keys = list(zip(base.pat_col.tolist(), base.pat_row.tolist()))
    new = (0, 4)
    keys2 = sorted(keys + [new])
    pos = keys2.index(new)
    inst = copy.deepcopy(base)
    inst.pat_col = np.array([k[0] for k in keys2], dtype=np.int32)
    inst.pat_row = np.array([k[1] for k in keys2], dtype=np.int32)
    inst.a_val = np.insert(base.a_val, pos, 0.0, axis=1)
    inst.c = np.insert(base.c, pos, 0.0)
    out.append(("uncovered", inst, -2))
    # a clique pair missing from the pattern
    inst = copy.deepcopy(base)
    drop = int(np.nonzero((base.pat_row == 1) & (base.pat_col == 0))[0][0])
    keep = np.array([j for j in range(base.nnz) if j != drop])
    inst.pat_row, inst.pat_col = base.pat_row[keep], base.pat_col[keep]
    inst.a_val, inst.c = base.a_val[:, keep], base.c[keep]
    out.append(("off_pattern", inst, -3))
    # clique vertices out of order
    inst = copy.deepcopy(base)
    cv = inst.clique_vert.copy()
    cv[0], cv[1] = cv[1], cv[0]
    inst.clique_vert = cv
    out.append(("clique_order", inst, -4))
    # non-finite data
    inst = copy.deepcopy(base)
    inst.c = base.c.copy()
    inst.c[2] = np.nan
    out.append(("nonfinite", inst, -6))
    # clique larger than 128
    out.append(("too_large", sdpgen.lovasz_theta_odd_cycle(129), -7))
    # unsorted pattern
    inst = copy.deepcopy(base)
    inst.pat_row = base.pat_row[::-1].copy()
    inst.pat_col = base.pat_col[::-1].copy()
    out.append(("unsorted_pattern", inst, -1))
    return out


def rank_deficient_instance():
    inst = sdpgen.block_arrow_instance(3, 3, 2, 5, seed=0)
    inst = copy.deepcopy(inst)
    inst.a_val = inst.a_val.copy()
    inst.a_val[3] = 2.0 * inst.a_val[1]
    return inst


def singleton_clique_instance(seed=3):
    """Block-arrow instance plus one isolated vertex (a clique of size 1)."""
    rng = np.random.default_rng(seed)
    cl = sdpgen.block_arrow_cliques(3, 4, 2)
    n = 3 * 4 + 2 + 1
    cl = cl + [np.array([n - 1], dtype=np.int32)]
    return sdpgen.random_instance(n, cl, 7, rng=rng, name="with_singleton")


def oracle_extended(inst):
    """The instance on the oracle's chordal extension of its pattern, with the
    oracle's maximal cliques (A and C zero on the added coordinates)."""
    from oracle import preprocess
    pr, pc, cl = preprocess.chordal_extension(inst.n, inst.pat_row, inst.pat_col)
    pos = {(int(r), int(c)): j for j, (r, c) in enumerate(zip(pr, pc))}
    idx = np.array([pos[(int(r), int(c))] for r, c in zip(inst.pat_row, inst.pat_col)])
    a = np.zeros((inst.m, pr.shape[0]))
    a[:, idx] = inst.a_dense()
    c = np.zeros(pr.shape[0])
    c[idx] = inst.c
    ptr, vert = sdpgen.cliques_to_csr([np.array(k, dtype=np.int32) for k in cl])
    return sdpgen.Instance(n=inst.n, m=inst.m, pat_row=pr, pat_col=pc, clique_ptr=ptr,
                           clique_vert=vert, a_format=sdpgen.A_DENSE, a_val=a, b=inst.b.copy(),
                           c=c, name=inst.name + "_ext")


def as_instance(d):
    """An sdpgen.Instance with the fields of any instance-like object."""
    return sdpgen.Instance(n=int(d.n), m=int(d.m), pat_row=d.pat_row, pat_col=d.pat_col,
                           clique_ptr=d.clique_ptr, clique_vert=d.clique_vert,
                           a_format=int(d.a_format), a_val=d.a_val, b=d.b, c=d.c,
                           a_rowptr=d.a_rowptr, a_col=d.a_col, name=getattr(d, "name", ""))
