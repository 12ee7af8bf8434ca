"""GPU parity of the standalone batched PSD projection against the oracle.

The kernel solves each block's eigenproblem by parallel-order Jacobi in LDS
and rebuilds V diag(max(theta, 0)) V^T; the oracle uses cyclic Jacobi in
FP64.  The projection is unique, so the outputs are compared element by
element: FP64 to 1e-11 ||W||_F, FP32 to 3e-5 ||W||_F (FP32 rounding of a
Jacobi eigensolver of size <= 128).
"""
import numpy as np
import pytest

import sdpgen

pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-11, np.float32: 3e-5}


def run_gpu(sdp, blocks, dtype, max_size, variant=None):
    import torch
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    sizes = np.array([b.shape[0] for b in blocks], dtype=np.int32)
    offs = np.concatenate([[0], np.cumsum(sizes.astype(np.int64) ** 2)[:-1]]).astype(np.int64)
    flat = np.concatenate([b.astype(dtype).ravel() for b in blocks])
    dev = torch.device("cuda:0")
    t_in = torch.from_numpy(flat).to(dev)
    t_out = torch.full_like(t_in, float("nan"))
    sdp.psd_project_batched(torch.from_numpy(sizes).to(dev), torch.from_numpy(offs).to(dev),
                            t_in, t_out, max_size, variant=variant)
    torch.cuda.synchronize()
    out = t_out.cpu().numpy().astype(np.float64)
    return [out[o:o + s * s].reshape(s, s) for o, s in zip(offs, sizes)]


def check(oracle_mod, blocks, outs, dtype):
    for W, X in zip(blocks, outs):
        Wd = W.astype(dtype).astype(np.float64)       # the input the kernel saw
        ref = oracle_mod.psd_project(0.5 * (Wd + Wd.T))
        scale = max(np.linalg.norm(Wd), 1e-300)
        err = np.abs(X - ref).max() / scale
        assert err <= TOL[dtype], (W.shape[0], err)
        assert np.array_equal(X, X.T)


CASES = [
    (np.float32, [1, 2, 3, 5, 8, 15, 16] * 3, 16),
    (np.float32, [17, 24, 31, 32] * 3, 32),
    (np.float32, [33, 50, 63, 64] * 2, 64),
    (np.float32, [65, 100, 127, 128], 128),
    (np.float64, [1, 2, 3, 5, 8, 15, 16] * 3, 16),
    (np.float64, [17, 24, 31, 32] * 3, 32),
    (np.float64, [33, 50, 63, 64] * 2, 64),
    (np.float64, [65, 80, 95, 96], 96),
]


@pytest.mark.parametrize("dtype,sizes,max_size", CASES,
                         ids=[f"{c[0].__name__}-{c[2]}" for c in CASES])
def test_projection_matches_oracle_goe(sdp, gpu, oracle_mod, dtype, sizes, max_size):
    print(f"projection dtype={dtype.__name__} max_size={max_size} sizes={sizes}", flush=True)
    blocks = sdpgen.goe_blocks(sizes, seed=max_size)
    outs = run_gpu(sdp, blocks, dtype, max_size)
    check(oracle_mod, blocks, outs, dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_every_kernel_variant_matches_oracle(sdp, gpu, oracle_mod, dtype):
    """Each (block size N, threads) variant the autotuner may pick, on sizes
    from the smallest that needs it to N, against the oracle."""
    dt = sdp.DTYPE_FP32 if dtype == np.float32 else sdp.DTYPE_FP64
    variants = sdp.projection_variants(dt)
    Ns = sorted({n for n, _ in variants})
    for v, (N, NT) in enumerate(variants):
        lo = max([n for n in Ns if n < N], default=0) + 1
        sizes = sorted({lo, (lo + N) // 2, N - 1, N}) + [1, 2]
        print(f"variant {v}: N={N} NT={NT} sizes={sizes}", flush=True)
        blocks = sdpgen.goe_blocks(sizes, seed=1000 + v)
        outs = run_gpu(sdp, blocks, dtype, N, variant=v)
        check(oracle_mod, blocks, outs, dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_projection_degenerate_inputs(sdp, gpu, oracle_mod, dtype):
    """Zero, PSD (fixed point), NSD (maps to 0), repeated and zero eigenvalues."""
    rng = np.random.default_rng(5)
    s = 12
    Q, _ = np.linalg.qr(rng.standard_normal((s, s)))
    G = rng.standard_normal((s, s))
    blocks = [
        np.zeros((s, s)),
        G @ G.T,                                    # PSD
        -(G @ G.T),                                 # NSD
        (Q * np.array([2.0] * 6 + [-1.0] * 6)) @ Q.T,   # repeated eigenvalues
        (Q * np.array([0.0] * 4 + [3.0] * 4 + [-3.0] * 4)) @ Q.T,
        np.diag(np.linspace(-2, 2, s)),
        np.eye(s) * 7.0,
    ]
    blocks = [0.5 * (b + b.T) for b in blocks]
    outs = run_gpu(sdp, blocks, dtype, 16)
    check(oracle_mod, blocks, outs, dtype)
    assert np.all(outs[0] == 0.0)
    assert np.all(np.abs(outs[2]) <= TOL[dtype] * np.linalg.norm(blocks[2]))


def test_projection_many_blocks_fill_the_chip(sdp, gpu, oracle_mod):
    """4096 blocks of 16 (more workgroups than CUs); spot-check a sample."""
    blocks = sdpgen.goe_blocks([16] * 4096, seed=11)
    outs = run_gpu(sdp, blocks, np.float32, 16)
    idx = np.random.default_rng(0).choice(4096, 64, replace=False)
    check(oracle_mod, [blocks[i] for i in idx], [outs[i] for i in idx], np.float32)


def test_projection_empty_call(sdp, gpu):
    import torch
    dev = torch.device("cuda:0")
    z32 = torch.zeros(0, dtype=torch.int32, device=dev)
    z64 = torch.zeros(0, dtype=torch.int64, device=dev)
    f = torch.zeros(0, dtype=torch.float32, device=dev)
    sdp.psd_project_batched(z32, z64, f, f.clone(), 16)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_sign_variants_degenerate_and_clustered_spectra(sdp, gpu, oracle_mod, dtype):
    """The sign-function variants (no eigenvectors) on zero, PSD, NSD,
    repeated and zero eigenvalues, and on spectra whose magnitudes spread
    log-uniformly down to 1e-9 (eigenvalues below the resolution contribute
    at most their size)."""
    dt = sdp.DTYPE_FP32 if dtype == np.float32 else sdp.DTYPE_FP64
    variants = sdp.projection_variants(dt)
    sign = [v for v in range(len(variants)) if sdp.projection_variant_kind(dt, v) == 2]
    assert sign, "no sign-function variants"
    rng = np.random.default_rng(9)
    for v in sign:
        N = variants[v][0]
        s = N - 3 if N > 16 else 12
        Q, _ = np.linalg.qr(rng.standard_normal((s, s)))
        G = rng.standard_normal((s, s))
        mags = 10 ** rng.uniform(-9, 0, s) * rng.choice([-1.0, 1.0], s)
        blocks = [np.zeros((s, s)), G @ G.T, -(G @ G.T),
                  (Q * np.array([2.0] * (s // 2) + [-1.0] * (s - s // 2))) @ Q.T,
                  (Q * np.concatenate([np.zeros(s // 3), 3.0 * np.ones(s // 3),
                                       -3.0 * np.ones(s - 2 * (s // 3))])) @ Q.T,
                  (Q * mags) @ Q.T, np.eye(s) * 7.0]
        blocks = [0.5 * (b + b.T) for b in blocks]
        print(f"sign variant {v}: N={N} s={s}", flush=True)
        outs = run_gpu(sdp, blocks, dtype, N, variant=v)
        check(oracle_mod, blocks, outs, dtype)
        assert np.all(outs[0] == 0.0)


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_nonfinite_blocks_give_nan_not_a_finite_result(sdp, gpu, dtype):
    """A block with a NaN or an infinite entry comes out all NaN from every
    variant (never zeros or a finite matrix); the other blocks of the batch
    are unaffected."""
    dt = sdp.DTYPE_FP32 if dtype == np.float32 else sdp.DTYPE_FP64
    variants = sdp.projection_variants(dt)
    rng = np.random.default_rng(2)
    good = 0.5 * (lambda G: G + G.T)(rng.standard_normal((10, 10)))
    bad_nan, bad_inf = good.copy(), good.copy()
    bad_nan[3, 4] = bad_nan[4, 3] = np.nan
    bad_inf[1, 1] = np.inf
    for v in [v for v in range(len(variants)) if variants[v][0] == 16]:
        outs = run_gpu(sdp, [good, bad_nan, bad_inf], dtype, 16, variant=v)
        print(f"variant {v} kind {sdp.projection_variant_kind(dt, v)}", flush=True)
        assert np.all(np.isfinite(outs[0]))
        assert np.all(np.isnan(outs[1])), outs[1]
        assert not np.any(np.isfinite(outs[2])), outs[2]


@pytest.mark.parametrize("dtype", [np.float32, np.float64], ids=["f32", "f64"])
def test_jacobi_variants_low_rank_and_definite_blocks(sdp, gpu, oracle_mod, dtype):
    """The eigenvector variants of blocks of 64 and more rebuild X from the
    positive eigenpairs only (a list of the positive slots): no positive
    eigenvalue (zero and negative definite blocks: X = 0), all of them
    (positive definite at the full size: X = W), rank 1, and rank 17 (the
    list crosses a 16-row tile), at s = N and s = N - 3."""
    dt = sdp.DTYPE_FP32 if dtype == np.float32 else sdp.DTYPE_FP64
    variants = sdp.projection_variants(dt)
    eig = [v for v in range(len(variants))
           if sdp.projection_variant_kind(dt, v) != 2 and variants[v][0] >= 64]
    assert eig, "no eigenvector variants of blocks of 64 and more"
    rng = np.random.default_rng(21)
    for v in eig:
        N = variants[v][0]
        for s in (N, N - 3):
            Q, _ = np.linalg.qr(rng.standard_normal((s, s)))
            G = rng.standard_normal((s, s))
            lam1 = -rng.uniform(0.5, 2.0, s)
            lam1[0] = 3.0
            lam17 = rng.uniform(-2.0, -0.1, s)
            lam17[rng.choice(s, 17, replace=False)] = rng.uniform(0.1, 2.0, 17)
            blocks = [np.zeros((s, s)), G @ G.T + s * np.eye(s), -(G @ G.T),
                      (Q * lam1) @ Q.T, (Q * lam17) @ Q.T]
            blocks = [0.5 * (b + b.T) for b in blocks]
            print(f"eigenvector variant {v}: N={N} NT={variants[v][1]} s={s}", flush=True)
            outs = run_gpu(sdp, blocks, dtype, N, variant=v)
            check(oracle_mod, blocks, outs, dtype)
            assert np.all(outs[0] == 0.0)
            assert np.all(np.abs(outs[2]) <= TOL[dtype] * np.linalg.norm(blocks[2]))
