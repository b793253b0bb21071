"""C-ABI contract, checked without a GPU.

The library must load, export every entry point include/dfmi.h declares, size
workspaces, and reject bad arguments with the documented status code before
it makes any HIP call (so these checks run on a machine with no device).
"""
import ctypes
import os
import re

import pytest

from paper_2505_03755_amd import dfmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "dfmi.h")).read()
    return sorted(set(re.findall(r"^\s*(?:df_status|const char\*)\s+(df_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(dfmi.LIB_PATH):
        pytest.skip("libdfmi.so not built")
    return dfmi.load_library()


@pytest.fixture()
def ctx(L):
    h = ctypes.c_void_p()
    assert L.df_create(ctypes.byref(h), 0, None) == dfmi.DF_OK
    yield h
    L.df_destroy(h)


def test_exports_every_declared_symbol(L):
    names = _header_functions()
    assert set(names) == set(dfmi.EXPORTED)
    for n in names:
        assert hasattr(L, n), n


def test_create_rejects_bad_arguments(L):
    assert L.df_create(None, 0, None) == dfmi.DF_ERR_ARG
    h = ctypes.c_void_p()
    assert L.df_create(ctypes.byref(h), -1, None) == dfmi.DF_ERR_ARG
    assert b"device" in L.df_last_error(None)
    assert L.df_destroy(None) == dfmi.DF_OK


def test_workspace_size(L):
    n = dfmi.workspace_size(dfmi.DF_OP_HALF_TRANSFORM, naux=10, nao=7, ncol=3)
    assert n >= 16 * 3 * 8          # C padded to 16 rows
    jk = dfmi.workspace_size(dfmi.DF_OP_JK, naux=10, nao=7, ndm=1, nocc=3)
    assert jk >= 10 * 7 * 3 * 8
    step = dfmi.workspace_size(dfmi.DF_OP_STEP, naux=10, nao=7, nocc=3, nac=2, np=7)
    assert step >= 10 * 7 * 5 * 8 + 10 * 7 * 2 * 8
    full = dfmi.workspace_size(dfmi.DF_OP_PAPA, naux=10, nao=7, nac=2, np=7, nq=5, flags=dfmi.DF_PAPA_FULL)
    assert full >= 10 * 5 * 2 * 8
    with pytest.raises(dfmi.DFError):
        dfmi.workspace_size(dfmi.DF_OP_JK, naux=0, nao=7, ndm=1, nocc=3)
    with pytest.raises(dfmi.DFError):
        dfmi.workspace_size(99, naux=10, nao=7)


P = ctypes.c_void_p


def fake(addr):
    """A pointer value that is never dereferenced: argument checks fail before any use."""
    return ctypes.c_void_p(addr)


def test_null_context(L):
    assert L.df_half_transform(None, fake(4096), 4, 3, fake(8192), 2, fake(16384), None, 0, None, 0) == dfmi.DF_ERR_ARG


def test_half_transform_argument_errors(L, ctx):
    B, C, X = fake(1 << 20), fake(2 << 20), fake(3 << 20)
    assert L.df_half_transform(ctx, None, 4, 3, C, 2, X, None, 0, None, 0) == dfmi.DF_ERR_ARG
    assert L.df_half_transform(ctx, B, 0, 3, C, 2, X, None, 0, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_half_transform(ctx, B, 4, -1, C, 2, X, None, 0, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_half_transform(ctx, B, 4, 3, C, 0, X, None, 0, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_half_transform(ctx, B, 4, 3, C, 2, X, None, 0, None, 7) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_half_transform(ctx, B, 4, 3, C, 2, X, fake(4 << 20), 3, None, 0) == dfmi.DF_ERR_ARG
    assert L.df_half_transform(ctx, B, 4, 3, C, 2, X, None, 3, None, 0) == dfmi.DF_ERR_SHAPE
    # output overlapping an input
    assert L.df_half_transform(ctx, B, 4, 3, C, 2, fake((1 << 20) + 8), None, 0, None, 0) == dfmi.DF_ERR_ARG
    assert b"overlaps" in L.df_last_error(ctx)
    # nao too large for 31-bit packed offsets
    assert L.df_half_transform(ctx, B, 4, 50000, C, 2, X, None, 0, None, 0) == dfmi.DF_ERR_SHAPE


def test_jk_argument_errors(L, ctx):
    B, C, J, K = fake(1 << 30), fake(2 << 30), fake(3 << 30), fake(4 << 30)
    assert L.df_jk(ctx, B, 10, 7, 0, C, 3, None, J, K, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_jk(ctx, B, 10, 7, 1, None, 3, None, J, K, None, 0) == dfmi.DF_ERR_ARG
    assert L.df_jk(ctx, B, 10, 7, 1, C, -2, None, J, K, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, 1) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, J, None, 0) == dfmi.DF_ERR_ARG   # J and K alias
    # no workspace attached
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, 0) == dfmi.DF_ERR_WORKSPACE
    need = dfmi.workspace_size(dfmi.DF_OP_JK, naux=10, nao=7, ndm=1, nocc=3)
    assert L.df_set_workspace(ctx, fake(5 << 30), need - 256) == dfmi.DF_OK
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_set_workspace(ctx, fake((5 << 30) + 8), need) == dfmi.DF_ERR_ARG  # misaligned
    assert L.df_set_workspace(ctx, fake((3 << 30)), need) == dfmi.DF_OK
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, 0) == dfmi.DF_ERR_ARG   # workspace overlaps J


def test_active_eri_and_papa_argument_errors(L, ctx):
    B, C, E = fake(1 << 30), fake(2 << 30), fake(3 << 30)
    assert L.df_active_eri(ctx, B, 10, 7, None, 2, E, None, 0) == dfmi.DF_ERR_ARG
    assert L.df_active_eri(ctx, B, 10, 7, C, -1, E, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_active_eri(ctx, B, 10, 7, C, 2, E, None, dfmi.DF_PAPA_FULL) == dfmi.DF_ERR_UNSUPPORTED
    # nac = 0: nothing to compute, no workspace needed, no device touched
    assert L.df_active_eri(ctx, B, 10, 7, None, 0, None, None, 0) == dfmi.DF_OK
    Cp, Ca, O = fake(4 << 30), fake(5 << 30), fake(6 << 30)
    assert L.df_papa(ctx, B, 10, 7, Cp, 7, Ca, 2, fake(7 << 30), 3, O, 0) == dfmi.DF_ERR_ARG   # Cq without FULL
    assert L.df_papa(ctx, B, 10, 7, Cp, 7, Ca, 2, None, 3, O, dfmi.DF_PAPA_FULL) == dfmi.DF_ERR_ARG
    assert L.df_papa(ctx, B, 10, 7, Cp, 7, Ca, 2, None, 0, O, 0x8) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_papa(ctx, B, 10, 7, Cp, 7, Ca, 2, None, 0, O, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_papa(ctx, B, 10, 7, Cp, 0, Ca, 2, None, 0, O, 0) == dfmi.DF_OK      # empty output


def test_ppaa_argument_errors(L, ctx):
    B, Cp, Cq, Ca, O = fake(1 << 30), fake(2 << 30), fake(3 << 30), fake(4 << 30), fake(5 << 30)
    assert L.df_ppaa(ctx, B, 10, 7, Cp, 7, Cq, 5, None, 2, O, 0) == dfmi.DF_ERR_ARG       # no Cact
    assert L.df_ppaa(ctx, B, 10, 7, Cp, 7, None, 5, Ca, 2, O, 0) == dfmi.DF_ERR_ARG       # nq without Cq
    assert L.df_ppaa(ctx, B, 10, 7, Cp, -1, None, 0, Ca, 2, O, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_ppaa(ctx, B, 10, 7, Cp, 7, None, 0, Ca, 2, O, 1) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_ppaa(ctx, B, 10, 7, Cp, 7, None, 0, Ca, 2, B, 0) == dfmi.DF_ERR_ARG       # out overlaps B
    assert L.df_ppaa(ctx, B, 10, 7, Cp, 7, None, 0, Ca, 2, O, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_ppaa(ctx, B, 10, 7, Cp, 7, None, 0, None, 0, None, 0) == dfmi.DF_OK      # nac = 0: empty
    # workspace: the packed b_uv, and W_uv [nuv][npair] plus W_uv Cq [nuv][nao][nq] for one chunk
    n = dfmi.workspace_size(dfmi.DF_OP_PPAA, naux=10, nao=7, nac=2, np=7)
    assert n >= (10 * 3 + 3 * 28 + 3 * 7 * 7) * 8
    assert dfmi.workspace_size(dfmi.DF_OP_PPAA, naux=10, nao=7, nac=2, np=7, nq=3) < n


def test_build_and_embed_argument_errors(L, ctx):
    M, E, Lo, B, info = fake(1 << 30), fake(2 << 30), fake(3 << 30), fake(4 << 30), fake(5 << 30)
    assert L.df_build_cholesky(ctx, M, E, 300, 20, Lo, B, None, 0) == dfmi.DF_ERR_ARG      # no info
    assert L.df_build_cholesky(ctx, M, E, 0, 20, Lo, B, info, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_build_cholesky(ctx, M, E, 300, 20, Lo, B, info, 1) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_build_cholesky(ctx, M, E, 300, 20, E, B, info, 0) == dfmi.DF_ERR_ARG       # L overlaps eri3
    assert L.df_build_cholesky(ctx, M, E, 300, 9000, Lo, B, info, 0) == dfmi.DF_ERR_SHAPE  # 128 npair >= 2^32
    assert L.df_build_cholesky(ctx, M, E, 300, 20, Lo, B, info, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_build_cholesky(ctx, M, E, 300, 20, M, E, info, 0) == dfmi.DF_ERR_WORKSPACE  # in place is allowed
    n = dfmi.workspace_size(dfmi.DF_OP_BUILD_CHOLESKY, naux=300, nao=20)
    assert n >= (3 * 128 * 128 + 300 * 128 + 128 * 210) * 8
    assert L.df_embed_cholesky(ctx, B, 30, 20, None, 5, E, 0) == dfmi.DF_ERR_ARG
    assert L.df_embed_cholesky(ctx, B, 30, 20, M, -1, E, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_embed_cholesky(ctx, B, 30, 20, M, 5, E, 2) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_embed_cholesky(ctx, B, 30, 20, M, 5, B, 0) == dfmi.DF_ERR_ARG              # Be overlaps B
    assert L.df_embed_cholesky(ctx, B, 30, 20, M, 5, E, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_embed_cholesky(ctx, B, 30, 20, None, 0, None, 0) == dfmi.DF_OK
    assert dfmi.workspace_size(dfmi.DF_OP_EMBED_CHOLESKY, naux=30, nao=20, ncol=5) >= 30 * 25 * 5 * 8


def test_step_argument_errors(L, ctx):
    B, Co, Ca, Cp = fake(1 << 30), fake(2 << 30), fake(3 << 30), fake(4 << 30)
    J, K = fake(5 << 30), fake(6 << 30)
    X = (None, None)
    assert L.df_step(ctx, B, 10, 7, None, 3, None, Ca, 2, Cp, 7, J, K, None, None, None, *X, 0) == dfmi.DF_ERR_ARG
    assert L.df_step(ctx, B, 10, 7, Co, 3, None, None, 2, Cp, 7, J, K, None, None, None, *X, 0) == dfmi.DF_ERR_ARG
    assert L.df_step(ctx, B, 10, 7, Co, 3, None, Ca, 2, Cp, 7, J, K, None, None, None, *X, 8) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_step(ctx, B, 10, 7, Co, 3, None, Ca, 2, Cp, 7, J, J, None, None, None, *X, 0) == dfmi.DF_ERR_ARG
    assert L.df_step(ctx, B, 10, 7, Co, 3, None, Ca, 2, Cp, 7, J, K, None, None, None, *X, 0) == dfmi.DF_ERR_WORKSPACE
    # Xocc and Xact come together
    assert L.df_step(ctx, B, 10, 7, Co, 3, None, Ca, 2, Cp, 7, J, K, None, None, None, fake(7 << 30), None, 0) == dfmi.DF_ERR_ARG
    # ... except that an empty one may be NULL: validation passes and the missing workspace is reported
    assert L.df_step(ctx, B, 10, 7, Co, 3, None, Ca, 0, Cp, 7, J, K, None, None, None, fake(7 << 30), None, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_step(ctx, B, 10, 7, Co, 0, None, Ca, 2, Cp, 7, J, K, None, None, None, None, fake(7 << 30), 0) == dfmi.DF_ERR_WORKSPACE
    # with caller-owned X the workspace shrinks by the two half transforms
    a = dfmi.workspace_size(dfmi.DF_OP_STEP, naux=10, nao=7, nocc=3, nac=2, np=7)
    b = dfmi.workspace_size(dfmi.DF_OP_STEP, naux=10, nao=7, nocc=3, nac=2, np=7, flags=dfmi.DF_CALLER_X)
    assert a - b >= 10 * 7 * 5 * 8


def test_step_backward_argument_errors(L, ctx):
    B, Co, Ca = fake(1 << 30), fake(2 << 30), fake(3 << 30)
    gJ, gK, dCo, dCa = fake(4 << 30), fake(5 << 30), fake(6 << 30), fake(7 << 30)
    f = L.df_step_backward
    assert f(ctx, B, 10, 7, None, 3, Ca, 2, gJ, gK, None, None, None, dCo, dCa, 0) == dfmi.DF_ERR_ARG
    assert f(ctx, B, 10, 7, Co, 3, Ca, 2, gJ, gK, None, None, None, None, dCa, 0) == dfmi.DF_ERR_ARG
    assert f(ctx, B, 10, 7, Co, 3, Ca, 2, gJ, gK, None, None, None, dCo, dCa, 1) == dfmi.DF_ERR_UNSUPPORTED
    assert f(ctx, B, 10, 7, Co, -3, Ca, 2, gJ, gK, None, None, None, dCo, dCa, 0) == dfmi.DF_ERR_SHAPE
    assert f(ctx, B, 10, 7, Co, 3, Ca, 2, gJ, gK, None, fake(8 << 30), None, dCo, dCa, 0) == dfmi.DF_ERR_ARG
    assert f(ctx, B, 10, 7, Co, 3, Ca, 0, gJ, gK, None, fake(8 << 30), None, dCo, None, 0) == dfmi.DF_ERR_WORKSPACE
    assert f(ctx, B, 10, 7, Co, 3, Ca, 2, gJ, gK, None, None, None, dCo, dCo, 0) == dfmi.DF_ERR_ARG   # outputs alias
    assert f(ctx, B, 10, 7, Co, 3, Ca, 2, gJ, gK, None, None, None, dCo, dCa, 0) == dfmi.DF_ERR_WORKSPACE
    w_all = dfmi.workspace_size(dfmi.DF_OP_STEP_BACKWARD, naux=10, nao=7, nocc=3, nac=2,
                                flags=dfmi.DF_BWD_GJ | dfmi.DF_BWD_GK | dfmi.DF_BWD_GERI)
    w_j = dfmi.workspace_size(dfmi.DF_OP_STEP_BACKWARD, naux=10, nao=7, nocc=3, nac=2, flags=dfmi.DF_BWD_GJ)
    assert w_all > w_j > 0


def test_valid_call_without_device_fails_loudly(L, ctx):
    """With arguments valid but no usable GPU, the first device call reports DF_ERR_HIP."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    B, C, X = fake(1 << 30), fake(2 << 30), fake(3 << 30)
    # without a workspace the call stops at the argument checks
    assert L.df_half_transform(ctx, B, 4, 3, C, 2, X, None, 0, None, 0) == dfmi.DF_ERR_WORKSPACE
    n = dfmi.workspace_size(dfmi.DF_OP_HALF_TRANSFORM, naux=4, nao=3, ncol=2)
    assert L.df_set_workspace(ctx, fake(4 << 30), n) == dfmi.DF_OK   # recorded only, never touched here
    st = L.df_half_transform(ctx, B, 4, 3, C, 2, X, None, 0, None, 0)
    assert st == dfmi.DF_ERR_HIP
    assert b"hipSetDevice" in L.df_last_error(ctx)
    assert L.df_set_workspace(ctx, None, 0) == dfmi.DF_OK


def test_split_argument_errors(L, ctx):
    A, B, C = fake(1 << 30), fake(2 << 30), fake(3 << 30)
    f = L.df_split_matmul
    assert f(ctx, A, 8, 4, B, 8, 5, 8, 3, C, 5, 0) == dfmi.DF_ERR_SHAPE          # nslice < 4
    assert f(ctx, A, 8, 4, B, 8, 5, 8, 9, C, 5, 0) == dfmi.DF_ERR_SHAPE          # nslice > 8
    assert f(ctx, A, 7, 4, B, 8, 5, 8, 7, C, 5, 0) == dfmi.DF_ERR_ARG            # lda < K
    assert f(ctx, A, 8, 4, B, 8, 5, 8, 7, C, 4, 0) == dfmi.DF_ERR_ARG            # ldc < N
    assert f(ctx, A, 8, 4, B, 8, 5, 8, 7, C, 5, 1) == dfmi.DF_ERR_UNSUPPORTED
    assert f(ctx, A, 8, 4, B, 8, 5, 8, 7, C, 5, 0) == dfmi.DF_ERR_WORKSPACE
    assert f(ctx, A, 8, 0, B, 8, 5, 8, 7, C, 5, 0) == dfmi.DF_OK                 # empty product
    Bs, Be = fake(4 << 30), fake(5 << 30)
    assert L.df_split_cholesky(ctx, B, 10, 7, 7, None, Be, 0) == dfmi.DF_ERR_ARG
    assert L.df_split_cholesky(ctx, B, 10, 7, 2, Bs, Be, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_split_cholesky(ctx, B, 10, 7, 7, fake((4 << 30) + 8), Be, 0) == dfmi.DF_ERR_ARG   # Bs unaligned
    s = L.df_step_split
    Co, Ca, Cp, J, K = fake(6 << 30), fake(7 << 30), fake(8 << 30), fake(9 << 30), fake(10 << 30)
    assert s(ctx, B, None, Be, 7, 10, 7, Co, 3, Ca, 2, Cp, 7, J, K, None, None, None, None, None, 0) == dfmi.DF_ERR_ARG
    assert s(ctx, B, Bs, Be, 7, 10, 7, None, 3, Ca, 2, Cp, 7, J, K, None, None, None, None, None, 0) == dfmi.DF_ERR_ARG
    assert s(ctx, B, Bs, Be, 3, 10, 7, Co, 3, Ca, 2, Cp, 7, J, K, None, None, None, None, None, 0) == dfmi.DF_ERR_SHAPE
    Bu = fake((4 << 30) + 8)
    assert s(ctx, B, Bu, Be, 7, 10, 7, Co, 3, Ca, 2, Cp, 7, J, K, None, None, None, None, None, 0) == dfmi.DF_ERR_ARG
    assert s(ctx, B, Bs, Be, 7, 10, 7, Co, 3, Ca, 2, Cp, 7, J, K, None, None, None, None, None, 0) == dfmi.DF_ERR_WORKSPACE


def test_split_adjoint_argument_errors(L, ctx):
    B, Bt, Bte = fake(1 << 30), fake(2 << 30), fake(3 << 30)
    Co, Ca, gK, Xo, Xa, dCo, dCa = (fake(k << 30) for k in range(4, 11))
    t = L.df_split_cholesky_t
    assert t(ctx, B, 10, 7, 7, None, Bte, 0) == dfmi.DF_ERR_ARG
    assert t(ctx, B, 10, 7, 3, Bt, Bte, 0) == dfmi.DF_ERR_SHAPE
    assert t(ctx, B, 10, 7, 7, fake((2 << 30) + 8), Bte, 0) == dfmi.DF_ERR_ARG      # Bt unaligned
    assert t(ctx, B, 10, 7, 7, Bt, Bte, 1) == dfmi.DF_ERR_UNSUPPORTED
    b = L.df_step_backward_split
    args = [ctx, B, Bt, Bte, 7, 10, 7, Co, 3, Ca, 2, None, gK, None, Xo, Xa, dCo, dCa, 0]
    assert b(*args) == dfmi.DF_ERR_WORKSPACE
    for i, code in ((2, dfmi.DF_ERR_ARG),        # gK without Bt
                    (14, dfmi.DF_ERR_ARG),       # gK without Xocc
                    (16, dfmi.DF_ERR_ARG)):      # nocc > 0 without dCocc
        bad = list(args)
        bad[i] = None
        assert b(*bad) == code
    bad = list(args)
    bad[4] = 9
    assert b(*bad) == dfmi.DF_ERR_SHAPE
    bad = list(args)
    bad[13] = fake(11 << 30)                      # geri without Xact
    bad[15] = None
    assert b(*bad) == dfmi.DF_ERR_ARG
    # Xocc and Xact of df_step_split go together
    s = L.df_step_split
    Bs, Be, Cp, J, K = fake(12 << 30), fake(13 << 30), fake(14 << 30), fake(15 << 30), fake(16 << 30)
    assert s(ctx, B, Bs, Be, 7, 10, 7, Co, 3, Ca, 2, Cp, 7, J, K, None, None, None, Xo, None, 0) == dfmi.DF_ERR_ARG
    w = dfmi.workspace_size(dfmi.DF_OP_STEP_BACKWARD_SPLIT, naux=20, nao=9, nocc=4, nac=2, nslice=7,
                            flags=dfmi.DF_BWD_GK)
    assert w >= 7 * 32 * 192 + 8 * 20 * 9 * 4   # planes of Y (rows i over (P, nu)) and Y itself (FP64)
    assert dfmi.workspace_size(dfmi.DF_OP_STEP_BACKWARD_SPLIT, naux=20, nao=9, nocc=4, nac=2, nslice=7) < w


def test_split_workspace_sizes():
    w = dfmi.workspace_size(dfmi.DF_OP_SPLIT_MATMUL, m=100, n=50, k=70, nslice=7)
    assert w >= 7 * (128 + 64) * 128 + 4 * 150         # planes: rows to 32, columns to 64; exponents
    assert dfmi.split_plane_shape(100, 70, 7) == (7, 4, 4, 1024)
    s5 = dfmi.workspace_size(dfmi.DF_OP_STEP_SPLIT, naux=20, nao=9, nocc=4, nac=2, np=9, nslice=5)
    s7 = dfmi.workspace_size(dfmi.DF_OP_STEP_SPLIT, naux=20, nao=9, nocc=4, nac=2, np=9, nslice=7)
    assert s7 > s5 > 0
    with pytest.raises(dfmi.DFError):
        dfmi.workspace_size(dfmi.DF_OP_STEP_SPLIT, naux=20, nao=9, nocc=4, nac=2, np=9, nslice=9)


def test_batched_argument_errors(L, ctx):
    P = dfmi.Problem
    arr = (P * 2)()
    arr[0] = P(1 << 30, 10, 7, 2, 2 << 30, 3, 3 << 30, 2, 4 << 30, 7, 5 << 30, 6 << 30, None, None)
    arr[1] = P(7 << 30, 12, 5, 1, 8 << 30, 2, None, 0, None, 0, 9 << 30, None, None, None)
    n = ctypes.c_size_t(0)
    assert L.df_batched_workspace_size(arr, 2, ctypes.byref(n)) == dfmi.DF_OK and n.value > 0
    assert L.df_batched_step(ctx, arr, 2, 1) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_batched_step(ctx, None, 2, 0) == dfmi.DF_ERR_ARG
    assert L.df_batched_step(ctx, arr, 2, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_batched_step(ctx, arr, 0, 0) == dfmi.DF_OK
    arr[1].J = 5 << 30                        # problem 1's J overlaps problem 0's J
    assert L.df_batched_step(ctx, arr, 2, 0) == dfmi.DF_ERR_ARG
    arr[1].J = 9 << 30
    arr[1].ndm = 0
    assert L.df_batched_step(ctx, arr, 2, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_batched_workspace_size(arr, 2, ctypes.byref(n)) == dfmi.DF_ERR_SHAPE
    arr[1].ndm = 1
    # (pq|uv): one more region, the size of problem 0's df_ppaa workspace
    assert L.df_batched_workspace_size(arr, 2, ctypes.byref(n)) == dfmi.DF_OK
    base = n.value
    arr[0].ppaa = 10 << 30
    assert L.df_batched_workspace_size(arr, 2, ctypes.byref(n)) == dfmi.DF_OK
    assert n.value - base == dfmi.workspace_size(dfmi.DF_OP_PPAA, naux=10, nao=7, nac=2, np=7)
    arr[0].Cp = None
    assert L.df_batched_step(ctx, arr, 2, 0) == dfmi.DF_ERR_ARG     # ppaa needs Cp
    arr[0].Cp = 4 << 30
    arr[0].ppaa = 5 << 30                     # overlaps problem 0's J
    assert L.df_batched_step(ctx, arr, 2, 0) == dfmi.DF_ERR_ARG


def test_batched_tuning_table(L, ctx):
    """The autotuning table: defaults, a stored choice per group shape, candidate checks."""
    P = dfmi.Problem
    arr = (P * 2)()
    arr[0] = P(1 << 30, 10, 7, 2, 2 << 30, 3, 3 << 30, 2, 4 << 30, 7, 5 << 30, 6 << 30, None, None)
    arr[1] = P(7 << 30, 12, 5, 1, 8 << 30, 2, None, 0, None, 0, 9 << 30, None, None, None)
    v = [ctypes.c_int(-1) for _ in range(4)]
    refs = [ctypes.byref(x) for x in v]

    def read():
        assert L.df_batched_tuning(ctx, arr, 2, *refs) == dfmi.DF_OK
        return tuple(x.value for x in v)

    assert read() == (176, 64, 16, 0)                      # defaults (N_ao <= 640: 64-wide K tiles)
    assert L.df_batched_set_tuning(ctx, arr, 2, 96, 128, 4) == dfmi.DF_OK
    assert read() == (96, 128, 4, 1)
    arr[0].ndm = 3                                        # another shape: defaults again
    assert read() == (176, 64, 16, 0)
    arr[0].ndm = 2
    assert read() == (96, 128, 4, 1)
    for bad in ((100, 128, 4), (96, 32, 4), (96, 128, 5)):
        assert L.df_batched_set_tuning(ctx, arr, 2, *bad) == dfmi.DF_ERR_ARG
    assert L.df_batched_tuning(ctx, arr, 2, None, refs[1], refs[2], refs[3]) == dfmi.DF_ERR_ARG
    assert L.df_set_autotune(None, 1) == dfmi.DF_ERR_ARG
    assert L.df_set_autotune(ctx, 1) == dfmi.DF_OK and L.df_set_autotune(ctx, 0) == dfmi.DF_OK


def test_batched_split_argument_errors(L, ctx):
    P = dfmi.Problem
    arr = (P * 2)()
    arr[0] = P(1 << 30, 10, 7, 2, 2 << 30, 3, 3 << 30, 2, 4 << 30, 7, 5 << 30, 6 << 30, None, None)
    arr[1] = P(7 << 30, 12, 5, 1, 8 << 30, 2, None, 0, None, 0, 9 << 30, None, None, None)
    bs = (ctypes.c_void_p * 2)(1 << 34, 2 << 34)
    be = (ctypes.c_void_p * 2)(3 << 34, 4 << 34)
    n = ctypes.c_size_t(0)
    assert L.df_batched_split_workspace_size(arr, 2, 7, 0, ctypes.byref(n)) == dfmi.DF_OK and n.value > 0
    w_split = n.value
    assert L.df_batched_split_workspace_size(arr, 2, 3, 0, ctypes.byref(n)) == dfmi.DF_ERR_SHAPE
    assert L.df_batched_split_workspace_size(arr, 2, 7, 1, ctypes.byref(n)) == dfmi.DF_ERR_UNSUPPORTED
    m = ctypes.c_size_t(0)
    assert L.df_batched_split_workspace_size(arr, 2, 7, dfmi.DF_SPLIT_K_FP64, ctypes.byref(m)) == dfmi.DF_OK
    assert 0 < m.value < w_split                   # no int8 copy of X_occ
    assert L.df_batched_step_split(ctx, arr, bs, be, 2, 7, 1) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_batched_step_split(ctx, arr, None, be, 2, 7, 0) == dfmi.DF_ERR_ARG
    assert L.df_batched_step_split(ctx, arr, bs, be, 2, 9, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_batched_step_split(ctx, arr, bs, be, 2, 7, 0) == dfmi.DF_ERR_WORKSPACE
    assert L.df_batched_step_split(ctx, arr, bs, be, 0, 7, 0) == dfmi.DF_OK
    bad = (ctypes.c_void_p * 2)((1 << 34) + 8, 2 << 34)                         # Bs not 16-byte aligned
    assert L.df_batched_step_split(ctx, arr, bad, be, 2, 7, 0) == dfmi.DF_ERR_ARG
    bad = (ctypes.c_void_p * 2)(1 << 34, None)
    assert L.df_batched_step_split(ctx, arr, bad, be, 2, 7, 0) == dfmi.DF_ERR_ARG


def test_accumulate_and_split_flags(L, ctx):
    """DF_ACCUMULATE and DF_PREC_SPLIT on the four calls: flag checks, the registration of the split of
    B per context and slice count, and the workspace each flag needs."""
    B, C, J, K = fake(1 << 30), fake(2 << 30), fake(3 << 30), fake(4 << 30)
    Bs, Be = fake(5 << 30), fake(6 << 30)
    SP, AC = dfmi.DF_PREC_SPLIT, dfmi.DF_ACCUMULATE
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, 0x8) == dfmi.DF_ERR_UNSUPPORTED
    # split precision without a registered split of B
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, SP) == dfmi.DF_ERR_ARG
    assert b"df_register_split" in L.df_last_error(ctx)
    assert L.df_half_transform(ctx, B, 10, 7, C, 2, J, None, 0, None, SP) == dfmi.DF_ERR_ARG
    assert L.df_active_eri(ctx, B, 10, 7, C, 2, J, None, SP) == dfmi.DF_ERR_ARG
    assert L.df_papa(ctx, B, 10, 7, C, 7, fake(7 << 30), 2, None, 0, J, SP) == dfmi.DF_ERR_ARG
    # registration checks
    reg = L.df_register_split
    assert reg(ctx, None, 10, 7, Bs, Be, 7) == dfmi.DF_ERR_ARG
    assert reg(ctx, B, 10, 7, Bs, Be, 3) == dfmi.DF_ERR_SHAPE
    assert reg(ctx, B, 10, 7, fake((5 << 30) + 8), Be, 7) == dfmi.DF_ERR_ARG       # Bs unaligned
    assert reg(ctx, B, 10, 7, Bs, None, 7) == dfmi.DF_ERR_ARG
    assert reg(ctx, B, 10, 7, Bs, Be, 7) == dfmi.DF_OK
    # registered: the call gets past the argument checks and stops at the missing workspace
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, SP) == dfmi.DF_ERR_WORKSPACE
    # the split planes are inputs: an output overlapping them is refused
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, fake((5 << 30) + 64), K, None, SP) == dfmi.DF_ERR_ARG
    # another slice count on the context: the 7-slice registration no longer applies
    assert L.df_set_split_slices(ctx, 9) == dfmi.DF_ERR_SHAPE
    assert L.df_set_split_slices(ctx, 5) == dfmi.DF_OK
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, SP) == dfmi.DF_ERR_ARG
    assert L.df_set_split_slices(ctx, 7) == dfmi.DF_OK
    assert reg(ctx, B, 10, 7, None, None, 7) == dfmi.DF_OK                          # removed
    assert L.df_jk(ctx, B, 10, 7, 1, C, 3, None, J, K, None, SP) == dfmi.DF_ERR_ARG
    for i in range(16):
        assert reg(ctx, fake((20 + i) << 30), 10, 7, Bs, Be, 7) == dfmi.DF_OK
    assert reg(ctx, fake(40 << 30), 10, 7, Bs, Be, 7) == dfmi.DF_ERR_ARG            # at most 16
    # accumulation with nothing to add (nocc = 0) touches nothing
    assert L.df_jk(ctx, B, 10, 7, 1, C, 0, None, J, K, None, AC) == dfmi.DF_OK
    # workspaces: the split forms need planes, accumulation with a second transform the new X
    ws = lambda op, **d: dfmi.workspace_size(op, **d)
    assert ws(dfmi.DF_OP_JK, naux=10, nao=7, ndm=2, nocc=3, flags=SP, nslice=7) > 0
    assert (ws(dfmi.DF_OP_JK, naux=10, nao=7, ndm=2, nocc=3, flags=SP | dfmi.DF_WEIGHTED, nslice=7)
            > ws(dfmi.DF_OP_JK, naux=10, nao=7, ndm=2, nocc=3, flags=SP, nslice=7))
    with pytest.raises(dfmi.DFError):
        ws(dfmi.DF_OP_JK, naux=10, nao=7, ndm=2, nocc=3, flags=SP)                 # nslice missing
    h0 = ws(dfmi.DF_OP_HALF_TRANSFORM, naux=10, nao=7, ncol=3, n2=4)
    assert ws(dfmi.DF_OP_HALF_TRANSFORM, naux=10, nao=7, ncol=3, n2=4, flags=AC) - h0 >= 10 * 7 * 3 * 8
    assert ws(dfmi.DF_OP_HALF_TRANSFORM, naux=10, nao=7, ncol=3, flags=AC) == ws(
        dfmi.DF_OP_HALF_TRANSFORM, naux=10, nao=7, ncol=3)
    # df_workspace_query takes the context's slice count for nslice = 0
    d = dfmi.Dims(naux=10, nao=7, nac=2, np=7, flags=SP)
    n = ctypes.c_size_t(0)
    assert L.df_workspace_query(ctx, dfmi.DF_OP_PAPA, ctypes.byref(d), ctypes.byref(n)) == dfmi.DF_OK
    assert n.value == ws(dfmi.DF_OP_PAPA, naux=10, nao=7, nac=2, np=7, flags=SP, nslice=7)
    assert L.df_set_split_slices(ctx, 5) == dfmi.DF_OK
    assert L.df_workspace_query(ctx, dfmi.DF_OP_PAPA, ctypes.byref(d), ctypes.byref(n)) == dfmi.DF_OK
    assert n.value == ws(dfmi.DF_OP_PAPA, naux=10, nao=7, nac=2, np=7, flags=SP, nslice=5)


def test_scratch_limit_chunks_the_adjoint(L, ctx):
    """df_set_scratch_limit: the adjoint's rows per chunk grow with the bound, the workspace stays
    within it, and a bound below one row is refused before any launch."""
    fl = dfmi.DF_BWD_GJ | dfmi.DF_BWD_GK | dfmi.DF_BWD_GERI
    dims = dict(naux=37, nao=50, nocc=6, nac=3, flags=fl)
    full = dfmi.workspace_size(dfmi.DF_OP_STEP_BACKWARD, **dims)
    d = dfmi.Dims(**dims)
    rows, n = ctypes.c_int64(0), ctypes.c_size_t(0)
    assert L.df_backward_chunk(ctx, ctypes.byref(d), ctypes.byref(rows)) == dfmi.DF_OK and rows.value == 37
    assert L.df_workspace_query(ctx, dfmi.DF_OP_STEP_BACKWARD, ctypes.byref(d), ctypes.byref(n)) == dfmi.DF_OK
    assert n.value == full
    last = 0
    for limit in (full * 3 // 10, full // 2, full * 7 // 10, full):
        assert L.df_set_scratch_limit(ctx, limit) == dfmi.DF_OK
        assert L.df_backward_chunk(ctx, ctypes.byref(d), ctypes.byref(rows)) == dfmi.DF_OK
        assert L.df_workspace_query(ctx, dfmi.DF_OP_STEP_BACKWARD, ctypes.byref(d), ctypes.byref(n)) == dfmi.DF_OK
        assert 1 <= rows.value <= 37 and n.value <= limit and rows.value >= last
        last = rows.value
    assert last == 37
    assert L.df_set_scratch_limit(ctx, 1024) == dfmi.DF_OK                          # below one row
    assert L.df_backward_chunk(ctx, ctypes.byref(d), ctypes.byref(rows)) == dfmi.DF_ERR_WORKSPACE
    assert L.df_workspace_query(ctx, dfmi.DF_OP_STEP_BACKWARD, ctypes.byref(d), ctypes.byref(n)) == dfmi.DF_ERR_WORKSPACE
    B, Co, Ca, gJ, gK, dCo, dCa = (fake(k << 30) for k in range(1, 8))
    assert L.df_step_backward(ctx, B, 37, 50, Co, 6, Ca, 3, gJ, gK, None, None, None, dCo, dCa, 0) == dfmi.DF_ERR_WORKSPACE
    assert b"scratch limit" in L.df_last_error(ctx)
    assert L.df_set_scratch_limit(ctx, 0) == dfmi.DF_OK


def test_jk_noalloc_argument_errors(L, ctx):
    B, C, J = fake(1 << 20), fake(1 << 30), fake(1 << 34)
    # only DF_ACCUMULATE is taken
    assert L.df_jk_noalloc(ctx, B, 8, 5, 1, C, 2, None, J, None, None, dfmi.DF_PREC_SPLIT) == dfmi.DF_ERR_UNSUPPORTED
    assert L.df_jk_noalloc(ctx, B, 8, 5, 0, C, 2, None, J, None, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_jk_noalloc(ctx, B, 8, 5, 1, C, -1, None, J, None, None, 0) == dfmi.DF_ERR_SHAPE
    assert L.df_jk_noalloc(ctx, None, 8, 5, 1, C, 2, None, J, None, None, 0) == dfmi.DF_ERR_ARG
    assert L.df_jk_noalloc(ctx, B, 8, 5, 1, None, 2, None, J, None, None, 0) == dfmi.DF_ERR_ARG
    # one auxiliary row of two densities at nao 3000 needs 2 * 3000^2 doubles of K partials: more
    # than the 128 MiB scratch, rejected before any HIP call
    st = L.df_jk_noalloc(ctx, B, 1, 3000, 2, C, 1, None, None, fake(1 << 40), None, 0)
    assert st == dfmi.DF_ERR_WORKSPACE
    assert b"static scratch" in L.df_last_error(ctx)
    # an output overlapping an input
    assert L.df_jk_noalloc(ctx, B, 8, 5, 1, C, 2, None, fake((1 << 20) + 64), None, None, 0) == dfmi.DF_ERR_ARG
    # nothing to add: returns before touching the device
    assert L.df_jk_noalloc(ctx, B, 8, 5, 1, C, 0, None, J, None, None, dfmi.DF_ACCUMULATE) == dfmi.DF_OK


def test_autotune_file_round_trip(L, tmp_path, monkeypatch):
    """The tuning table written to a file, read back into another context, and picked up at creation
    through DFMI_AUTOTUNE_CACHE; bad files are refused, foreign entries skipped."""
    import json
    P = dfmi.Problem
    arr = (P * 2)()
    arr[0] = P(1 << 30, 10, 7, 2, 2 << 30, 3, 3 << 30, 2, 4 << 30, 7, 5 << 30, 6 << 30, None, None)
    arr[1] = P(7 << 30, 12, 5, 1, 8 << 30, 2, None, 0, None, 0, 9 << 30, None, None, None)
    v = [ctypes.c_int(-1) for _ in range(4)]
    refs = [ctypes.byref(x) for x in v]

    def new_ctx():
        h = ctypes.c_void_p()
        assert L.df_create(ctypes.byref(h), 0, None) == dfmi.DF_OK
        return h

    def read(h):
        assert L.df_batched_tuning(h, arr, 2, *refs) == dfmi.DF_OK
        return tuple(x.value for x in v)

    monkeypatch.delenv("DFMI_AUTOTUNE_CACHE", raising=False)
    a = new_ctx()
    assert L.df_batched_set_tuning(a, arr, 2, 48, 128, 64) == dfmi.DF_OK
    path = str(tmp_path / "tune.json")
    assert L.df_autotune_save(a, path.encode()) == dfmi.DF_OK
    doc = json.load(open(path))
    assert doc["format"] == "dfmi-autotune/1"
    (e,) = doc["entries"]
    assert e["op"] == "df_batched_step" and e["precision"] == "fp64" and e["arch"] == ""
    assert (e["half_tile_n"], e["k_tile"], e["k_rounds"]) == (48, 128, 64)
    b = new_ctx()
    assert read(b) == (176, 64, 16, 0)
    assert L.df_autotune_load(b, path.encode()) == dfmi.DF_OK
    assert read(b) == (48, 128, 64, 1)
    # entries of another operation, precision or architecture, or outside the candidates, are skipped
    doc["entries"] += [dict(e, op="df_step"), dict(e, precision="split", half_tile_n=96),
                       dict(e, arch="gfx999", k_tile=64), dict(e, shape=e["shape"] + "x", k_rounds=5)]
    doc["entries"][0]["k_rounds"] = 4
    other = str(tmp_path / "other.json")
    json.dump(doc, open(other, "w"))
    c = new_ctx()
    assert L.df_autotune_load(c, other.encode()) == dfmi.DF_OK
    assert read(c) == (48, 128, 4, 1)
    # the environment variable: loaded at creation
    monkeypatch.setenv("DFMI_AUTOTUNE_CACHE", path)
    d = new_ctx()
    assert read(d) == (48, 128, 64, 1)
    # refused: a missing file, a file in another format (also through the environment), an empty path
    assert L.df_autotune_load(c, str(tmp_path / "none.json").encode()) == dfmi.DF_ERR_ARG
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": []}')
    assert L.df_autotune_load(c, str(bad).encode()) == dfmi.DF_ERR_ARG
    assert b"dfmi-autotune/1" in L.df_last_error(c)
    monkeypatch.setenv("DFMI_AUTOTUNE_CACHE", str(bad))
    h = ctypes.c_void_p()
    assert L.df_create(ctypes.byref(h), 0, None) == dfmi.DF_ERR_ARG
    assert b"DFMI_AUTOTUNE_CACHE" in L.df_last_error(None)
    monkeypatch.delenv("DFMI_AUTOTUNE_CACHE")
    assert L.df_autotune_save(c, b"") == dfmi.DF_ERR_ARG
    assert L.df_autotune_save(c, str(tmp_path / "no" / "dir.json").encode()) == dfmi.DF_ERR_ARG
    for h in (a, b, c, d):
        L.df_destroy(h)
