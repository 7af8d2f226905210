"""Device memory through the caller's allocator (bf_alloc): with the binding's
torch-backed allocator, a construction's workspace and factor storage are
torch's own blocks (visible in torch.cuda.memory_allocated and returned when
the factors are freed), results are bitwise those of the library's pool, and
freeing factors while an apply still runs on another stream never hands their
memory to a new construction too early."""
import sys

import numpy as np
import pytest

import workloads as wl

pytestmark = pytest.mark.gpu


def _same_bits(a, b):
    """Bitwise equality of two complex64 device tensors (any strides)."""
    x = np.ascontiguousarray(a.cpu().numpy()).view(np.uint32)
    y = np.ascontiguousarray(b.cpu().numpy()).view(np.uint32)
    return x.shape == y.shape and np.array_equal(x, y)


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


@pytest.fixture(scope="module")
def seg(bf):
    g = wl.segment_pair(4096, ppw=8.0)
    return bf.segkernel(g.targets, g.sources, g.k)


def test_torch_allocator_accounts_for_the_construction(bf, seg):
    import torch
    A = bf.torch_allocator()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    live0 = A.live_blocks()
    torch.cuda.reset_peak_memory_stats()
    say("construct n=4096 with the torch allocator")
    F = bf.construct(seg, 1e-6, 64, seed=21, allocator="torch")
    torch.cuda.synchronize()
    st = F.stats()
    held = torch.cuda.memory_allocated() - base
    peak = torch.cuda.max_memory_allocated() - base
    say(f"factors {st.device_bytes} B, torch holds {held} B, peak {peak} B")
    # the factor storage is torch's, and the workspace came on top of it
    assert held >= st.device_bytes > 0
    assert peak > held
    assert A.live_blocks() > live0
    F.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == base
    assert A.live_blocks() == live0


def test_library_pool_is_not_torch_memory(bf, seg):
    import torch
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    F = bf.construct(seg, 1e-6, 64, seed=21, allocator=None)
    torch.cuda.synchronize()
    assert torch.cuda.max_memory_allocated() == base
    F.close()


def test_allocators_give_bitwise_equal_results(bf, seg):
    import torch
    Fa = bf.construct(seg, 1e-6, 64, seed=22, allocator="torch")
    Fb = bf.construct(seg, 1e-6, 64, seed=22, allocator=None)
    assert np.array_equal(Fa.export().view(np.uint64), Fb.export().view(np.uint64))
    X = torch.from_numpy(wl.test_columns(4096, 24, 5).astype(np.complex64)).cuda()
    for trans in (False, True):
        ya = Fa.apply(X, trans=trans, allocator="torch")
        yb = Fb.apply(X, trans=trans, allocator=None)
        torch.cuda.synchronize()
        assert _same_bits(ya, yb)
    Fa.close()
    Fb.close()


@pytest.mark.parametrize("allocator", ["torch", None])
def test_close_while_applying_on_a_side_stream(bf, seg, allocator):
    """Factors closed (default stream) while a 256-column apply still reads
    them on a side stream; a new construction right after must not receive
    their blocks before that apply is done."""
    import torch
    X = torch.from_numpy(wl.test_columns(4096, 256, 9).astype(np.complex64)).cuda()
    F = bf.construct(seg, 1e-6, 64, seed=23, allocator=allocator)
    ref = F.apply(X)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        Y = F.apply(X, allocator=allocator)
    F.close()
    say(f"closed during a side-stream apply (allocator={allocator}); construct again")
    G = bf.construct(seg, 1e-6, 64, seed=24, allocator=allocator)
    torch.cuda.synchronize()
    assert _same_bits(Y, ref)
    G.close()


def test_server_with_torch_allocator(bf, seg):
    """The request engine takes every request's memory from torch's allocator
    (constructions and merged applies) and returns it when torn down."""
    import torch
    A = bf.torch_allocator()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    live0 = A.live_blocks()
    S = bf.Server(slots=2, batch_cols=16, allocator="torch")
    tc = S.submit_construct(seg, 1e-6, 64, seed=25)
    xs = [torch.from_numpy(wl.test_columns(4096, 2, 30 + i).astype(np.complex64)).cuda()
          for i in range(4)]
    ta = [S.submit_apply(tc, x) for x in xs]
    for t in [tc] + ta:
        S.wait(t)
    F = S.factors(tc)
    assert torch.cuda.memory_allocated() - base >= F.stats().device_bytes
    ys = [S.result(t) for t in ta]
    for x, y in zip(xs, ys):
        ref = F.apply(x, allocator=None)
        torch.cuda.synchronize()
        assert float((y - ref).norm() / ref.norm()) < 1e-6
    S.close()
    torch.cuda.synchronize()
    assert A.live_blocks() == live0
