"""The allocation-free force entry point (ihmc_force_noalloc) against the
existing one (ihmc_force): same force pass, so the same bits, on two calls in a
row (the second on a smaller lattice, over the first call's scratch
contents), in 2D and 3D, FP32 and FP64, without and with a uniform field, on
the context stream and on a caller's stream.  Device arrays come from torch;
the entry point itself allocates nothing."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1912_03278_amd import ihmc
    c = ihmc.Context(arena_bytes=256 << 20)
    yield c
    c.close()


def _noalloc(ctx, lat, psi, prec, on_torch_stream):
    """The force through the allocation-free entry point, on the context stream
    (synchronised on both sides), or on a stream of torch's (the ordering of
    torch's work and the library's then comes from the stream itself; torch's
    default stream has the handle 0, which the entry point reads as "the
    context stream", so a stream of its own is made)."""
    import torch
    dt = torch.float32 if prec == 4 else torch.float64
    if on_torch_stream:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            x = torch.tensor(psi, dtype=dt, device="cuda")
            F = torch.full_like(x, float("nan"))
            assert s.cuda_stream != 0
            ctx.force_noalloc(lat, x.data_ptr(), F.data_ptr(), precision=prec, stream=s.cuda_stream)
            out = F.cpu().numpy().astype(np.float64)
        return out
    x = torch.tensor(psi, dtype=dt, device="cuda")
    F = torch.full_like(x, float("nan"))
    torch.cuda.synchronize()
    ctx.force_noalloc(lat, x.data_ptr(), F.data_ptr(), precision=prec)
    ctx.sync()
    return F.cpu().numpy().astype(np.float64)


CASES = [
    ("2d", [((200, 150), 0.44, 4.1, None), ((70, 19), 0.4, 4.3, 0.05)]),
    ("3d", [((40, 30, 20), 0.22, 6.1, 0.02), ((9, 7, 5), 0.3, 6.5, None)]),
]


@pytest.mark.parametrize("prec", [4, 8])
@pytest.mark.parametrize("name,pair", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("on_torch_stream", [False, True])
def test_noalloc_force_equals_force(ctx, prec, name, pair, on_torch_stream):
    from paper_1912_03278_amd import ihmc
    rng = np.random.default_rng(1)
    for L, beta, C, h in pair:  # two calls in a row, the second smaller
        N = int(np.prod(L))
        psi = rng.standard_normal(N)
        psi = psi.astype(np.float32).astype(np.float64) if prec == 4 else psi
        lat = ihmc.Lattice(L, beta=beta, C=C, h=h)
        got = _noalloc(ctx, lat, psi, prec, on_torch_stream)
        ref = ctx.force(lat, psi, precision=prec)
        assert np.array_equal(got, ref), (L, np.max(np.abs(got - ref)))


def test_noalloc_force_against_oracle(ctx, orc):
    from paper_1912_03278_amd import ihmc
    psi = np.random.default_rng(2).standard_normal(33 * 21)
    lat = ihmc.Lattice((33, 21), beta=0.45, C=4.1, h=0.1)
    got = _noalloc(ctx, lat, psi, 8, False)
    ref = orc.force(orc.Lattice((33, 21), beta=0.45, C=4.1, h=0.1), psi)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_noalloc_force_refusals(ctx):
    import torch
    from paper_1912_03278_amd import ihmc
    x = torch.zeros(16, dtype=torch.float32, device="cuda")
    with pytest.raises(ihmc.IhmcError) as e:  # per-site field
        ctx.force_noalloc(ihmc.Lattice((4, 4), beta=0.4, C=4.1, h=np.zeros(16)), x.data_ptr(), x.data_ptr())
    assert e.value.code == -6
    with pytest.raises(ihmc.IhmcError) as e:  # beyond the 32 MiB scratch: checked before any launch
        ctx.force_noalloc(ihmc.Lattice((2048, 2048), beta=0.4, C=4.1), x.data_ptr(), x.data_ptr())
    assert e.value.code == -1
    with pytest.raises(ihmc.IhmcError) as e:
        ctx.force_noalloc(ihmc.Lattice((4, 4), beta=0.4, C=3.9), x.data_ptr(), x.data_ptr())
    assert e.value.code == -1
    # the entry point still works after the refusals
    lat = ihmc.Lattice((8, 8), beta=0.4, C=4.1)
    psi = np.random.default_rng(3).standard_normal(64).astype(np.float32).astype(np.float64)
    assert np.array_equal(_noalloc(ctx, lat, psi, 4, False), ctx.force(lat, psi, precision=4))
