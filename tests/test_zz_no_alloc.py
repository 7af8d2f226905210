"""bf_apply_noalloc (the apply whose intermediates live in the library's fixed
per-device scratch array) against bf_apply, through the C ABI: same kernels,
so the results must agree bit for bit, on consecutive calls whose sizes shrink
and at the largest column count the scratch holds; an oversized call is
rejected before anything is launched."""
import ctypes as C
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bf():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2002_03400_amd as m
    m.lib()
    return m


def _factors(bf, n, seed):
    g = wl.segment_pair(n, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say(f"construct n={n} seed={seed}")
    return op, bf.construct(op, 1e-6, 64, seed=seed)


def _tmp_rows(F):
    """Largest rank sum over the levels (rows of one ping-pong intermediate)."""
    kU, kV = F.ranks()
    return int(max(kU.sum(axis=1).max(), kV.sum(axis=1).max()))


def _pair(bf, F, trans, ncols, seed):
    """(bf_apply result, bf_apply_noalloc result, return code) for ncols columns."""
    import torch
    rows_in, rows_out = (F.m, F.n) if trans else (F.n, F.m)
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((ncols, rows_in)) + 1j * rng.standard_normal((ncols, rows_in)))
    Xd = torch.from_numpy(X.astype(np.complex64)).cuda().t()          # column-major view
    Y0 = torch.full((ncols, rows_out), 7.0 + 7.0j, dtype=torch.complex64, device="cuda").t()
    Y1 = torch.full((ncols, rows_out), 7.0 + 7.0j, dtype=torch.complex64, device="cuda").t()
    s = torch.cuda.current_stream().cuda_stream
    lib = bf.lib()
    say(f"apply n={F.n} trans={trans} ncols={ncols}")
    rc0 = lib.bf_apply(F._h, trans, Xd.data_ptr(), rows_in, ncols, Y0.data_ptr(), rows_out,
                       None, s)
    assert rc0 == 0, bf.lib().bf_last_error()
    rc1 = lib.bf_apply_noalloc(F._h, trans, Xd.data_ptr(), rows_in, ncols, Y1.data_ptr(),
                               rows_out, s)
    torch.cuda.synchronize()
    return Y0.cpu().numpy(), Y1.cpu().numpy(), rc1


def test_noalloc_matches_apply_on_shrinking_calls(bf):
    op, F = _factors(bf, 4096, 11)
    for trans in (0, 1):
        for ncols in (40, 3, 1):            # each call smaller than the one before
            Y0, Y1, rc = _pair(bf, F, trans, ncols, 100 * trans + ncols)
            assert rc == 0, bf.lib().bf_last_error()
            assert np.isfinite(Y0).all()
            assert np.array_equal(Y0.view(np.uint64), Y1.view(np.uint64)), (trans, ncols)
    # a second, smaller factorization reuses the same scratch array
    op2, F2 = _factors(bf, 2048, 12)
    for trans in (0, 1):
        Y0, Y1, rc = _pair(bf, F2, trans, 5, 7 + trans)
        assert rc == 0, bf.lib().bf_last_error()
        assert np.array_equal(Y0.view(np.uint64), Y1.view(np.uint64)), trans
    F2.close()
    F.close()


def test_noalloc_largest_and_oversized_calls(bf):
    op, F = _factors(bf, 2048, 13)
    cap = int(bf.lib().bf_apply_noalloc_scratch_bytes())
    assert cap == 64 << 20
    t = _tmp_rows(F)
    # two intermediates of t x ncols complex64, the second 256-byte aligned
    fits = lambda c: ((t * c * 8 + 255) // 256) * 256 + t * c * 8 <= cap
    big = (cap - 256) // (16 * t)
    while fits(big + 1):
        big += 1
    assert fits(big) and not fits(big + 1)
    say(f"tmp_rows={t} largest ncols={big}")
    Y0, Y1, rc = _pair(bf, F, 0, big, 21)
    assert rc == 0, bf.lib().bf_last_error()
    assert np.array_equal(Y0.view(np.uint64), Y1.view(np.uint64))
    Y0, Y1, rc = _pair(bf, F, 1, big + 1, 22)
    assert rc == -1
    assert b"scratch" in bf.lib().bf_last_error()
    assert np.all(Y1 == np.complex64(7 + 7j))        # nothing was launched
    F.close()
