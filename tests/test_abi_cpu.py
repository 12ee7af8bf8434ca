"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point include/sdp.h declares, its structs have the header's
layout, and the validation layer returns the same status codes as the oracle
(validation runs before any device call)."""
import os
import re
import subprocess

import numpy as np
import pytest

import sdpgen
from cases import invalid_instances

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sdp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sdp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(sdp):
    names = declared_functions()
    assert len(names) >= 13
    for n in names:
        assert hasattr(sdp.lib, n), n
    assert set(names) == set(sdp.EXPORTS)
    out = subprocess.check_output(["nm", "-D", "--defined-only", sdp.lib._name], text=True)
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def test_struct_layout_matches_header(sdp, tmp_path):
    import ctypes as C
    from paper_1707_05058_amd import _native as nat
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sdp.h"', 'int main(void){']
    for st in (nat.sdp_instance, nat.sdp_options, nat.sdp_result):
        lines.append(f'printf("{st.__name__} %zu\\n", sizeof({st.__name__}));')
        for f, _ in st._fields_:
            lines.append(f'printf("{st.__name__}.{f} %zu\\n", offsetof({st.__name__}, {f}));')
    lines.append("return 0;}")
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)], text=True).splitlines())
    for st in (nat.sdp_instance, nat.sdp_options, nat.sdp_result):
        assert int(got[st.__name__]) == C.sizeof(st)
        for f, _ in st._fields_:
            assert int(got[f"{st.__name__}.{f}"]) == getattr(st, f).offset, f


def test_default_options(sdp):
    o = sdp.default_options()
    assert o.rho == 1.0 and o.tol == 1e-4 and o.max_iter == 20000
    assert o.precision == sdp.FP64 and o.adaptive_rho == 0
    assert o.mu == 2.0 and o.nu == 10.0 and o.rho_period == 1 and o.graph_chunk > 0


@pytest.mark.parametrize("case", invalid_instances(), ids=lambda c: c[0])
def test_validation_codes_match_oracle(sdp, oracle_mod, case):
    name, inst, code = case
    assert oracle_mod.create_status(inst) == code
    assert sdp.setup_status([inst]) == code


def test_invalid_options_rejected(sdp):
    inst = sdpgen.block_arrow_instance(2, 2, 1, 3, seed=0)
    assert sdp.setup_status([inst], rho=-1.0) == -1
    assert sdp.setup_status([inst], max_iter=0) == -1
    assert sdp.setup_status([inst], precision=7) == -1


def test_projection_size_limits(sdp):
    """Blocks of up to 128 in both precisions and every algorithm (host
    checks, before any device work)."""
    for prec in (sdp.FP64, sdp.FP32_EIG):
        for alg in ("primal", "dual", "hsde"):
            assert sdp.setup_status([sdpgen.lovasz_theta_odd_cycle(129)], precision=prec,
                                    algorithm=alg) == -7
            assert "128" in sdp.lib.sdp_last_error().decode()


def test_batch_error_names_instance(sdp):
    good = sdpgen.block_arrow_instance(2, 2, 1, 3, seed=0)
    bad = invalid_instances()[2][1]
    assert sdp.setup_status([good, bad]) == -4
    assert "instance 1" in sdp.lib.sdp_last_error().decode()


def test_projection_argument_checks(sdp):
    import ctypes as C
    lib = sdp.lib
    assert lib.sdp_psd_project_batched(0, 16, None, None, None, None, 0, None) == 0
    assert lib.sdp_psd_project_batched(-1, 16, None, None, None, None, 0, None) == -1
    assert lib.sdp_psd_project_batched(0, 16, None, None, None, None, 5, None) == -1
    assert lib.sdp_psd_project_batched(0, 129, None, None, None, None, 1, None) == -7
    assert lib.sdp_psd_project_batched(0, 129, None, None, None, None, 0, None) == -7
    assert lib.sdp_psd_project_batched(0, 128, None, None, None, None, 0, None) == 0
    # explicit variants: index range, block size that must hold max_size
    v32 = sdp.projection_variants(sdp.DTYPE_FP32)
    v64 = sdp.projection_variants(sdp.DTYPE_FP64)
    assert max(n for n, _ in v32) == 128 and max(n for n, _ in v64) == 128
    for n, nt in v32 + v64:
        assert n % 16 == 0 and nt % 64 == 0 and (n // 2) ** 2 % nt == 0
    assert lib.sdp_psd_project_variant(-1, 0, 16, None, None, None, None, 1, None) == -1
    assert lib.sdp_psd_project_variant(len(v32), 0, 16, None, None, None, None, 1, None) == -1
    small = [i for i, (n, _) in enumerate(v32) if n == 16][0]
    assert lib.sdp_psd_project_variant(small, 0, 16, None, None, None, None, 1, None) == 0
    assert lib.sdp_psd_project_variant(small, 0, 17, None, None, None, None, 1, None) == -1
    assert lib.sdp_projection_variants(7, 0, None, None, None) == -1


def test_null_handle_is_rejected(sdp):
    assert sdp.lib.sdp_reset(None) == -1
    assert sdp.lib.sdp_admm_step(None, 1, None) == -1
    assert sdp.lib.sdp_get_stats(None, None, None) == -1


def test_projection_variant_kinds(sdp):
    """Every listed variant reports its method; the two-level ones have
    blocks of at least 64 (16 x 16 pair problems of groups of 8)."""
    for dt in (sdp.DTYPE_FP32, sdp.DTYPE_FP64):
        vs = sdp.projection_variants(dt)
        kinds = [sdp.projection_variant_two_level(dt, v) for v in range(len(vs))]
        assert any(kinds) and not all(kinds)
        for (N, NT), k in zip(vs, kinds):
            if k:
                assert N >= 64 and N % 16 == 0 and NT >= 64 * (N // 16)
    import ctypes as C
    t = C.c_int32(0)
    assert sdp.lib.sdp_projection_variant_kind(sdp.DTYPE_FP32, -1, C.byref(t)) == -1
    assert sdp.lib.sdp_projection_variant_kind(sdp.DTYPE_FP32, len(sdp.projection_variants(sdp.DTYPE_FP32)),
                                               C.byref(t)) == -1
    assert sdp.lib.sdp_projection_variant_kind(7, 0, C.byref(t)) == -1


@pytest.mark.parametrize("dtype_name", ["DTYPE_FP32", "DTYPE_FP64"])
def test_standalone_default_is_the_register_kernel_up_to_32(sdp, dtype_name):
    """sdp_psd_project_batched's default for blocks of up to 32 is the one-wave
    sign-function kernel (N = 16 up to 16, N = 32 for 17..32, 64 threads),
    which measured 1.6x faster than the LDS variant of 32 on 4096 blocks;
    above 32, the sign variant of the smallest fitting N."""
    dt = getattr(sdp, dtype_name)
    variants = sdp.projection_variants(dt)
    for s in range(1, 33):
        v = sdp.projection_default_variant(dt, s)
        N, NT = variants[v]
        assert sdp.projection_variant_kind(dt, v) == 2
        assert (N, NT) == ((16, 64) if s <= 16 else (32, 64)), (s, N, NT)
    nmax = max(n for n, _ in variants)
    for s in range(33, nmax + 1):
        v = sdp.projection_default_variant(dt, s)
        N, _ = variants[v]
        assert sdp.projection_variant_kind(dt, v) == 2
        assert N == min(n for n, _ in variants if n >= s + (s & 1))
    with pytest.raises(sdp.SdpError):
        sdp.projection_default_variant(dt, nmax + 1)
