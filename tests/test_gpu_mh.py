"""Checkerboard Metropolis-Hastings on the GPU (the comparison method of Sec. 4)
against the oracle's: the acceptance probabilities are tabulated on the host
with the oracle's own expression and every uniform is the same Philox draw,
so spins, m and beta*eps after every sweep must be identical, bit for bit;
statistics against enumeration."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1912_03278_amd import ihmc
    c = ihmc.Context(arena_bytes=512 << 20)
    yield c
    c.close()


@pytest.mark.parametrize("L,beta,h", [((64, 48), 0.44, 0.0), ((30, 10), 0.5, 0.03), ((8, 6, 10), 0.22, 0.0),
                                      ((2, 4), 0.3, 0.1), ((16, 16, 16), 0.2216544, 0.01)])
@pytest.mark.parametrize("given", [False, True])
def test_mh_bitwise_equal_to_oracle(ctx, orc, L, beta, h, given):
    from paper_1912_03278_amd import ihmc
    N = int(np.prod(L))
    s0 = np.where(np.random.default_rng(1).random(N) < 0.7, 1, -1).astype(np.int8) if given else None
    g = ctx.mh_run(ihmc.Lattice(L, beta=beta, C=2 * len(L) + 0.1, h=h if h else None), 40, seed=7, chain_id=3,
                   spins0=s0)
    r = orc.mh_run(orc.Lattice(L, beta=beta, C=2 * len(L) + 0.1, h=h if h else None), 40, seed=7, chain_id=3,
                   spins0=s0)
    assert np.array_equal(g["spins"], r["spins"])
    assert np.array_equal(g["m"], r["m"]) and np.array_equal(g["beta_eps"], r["beta_eps"])
    assert g["acceptance"] == r["acceptance"]


def test_mh_statistics_4x4(ctx):
    from paper_1912_03278_amd import ihmc
    from oracle import exact as E
    from oracle import stats as S
    ex = E.brute_force(E.torus_adjacency((4, 4)), 0.4, h=0.1)
    g = ctx.mh_run(ihmc.Lattice((4, 4), beta=0.4, C=4.1, h=0.1), 100000, seed=2)
    for key, series in (("be", g["beta_eps"]), ("m", g["m"]), ("m2", g["m"] ** 2)):
        st = S.gamma_method(series[100:])
        assert abs(st["mean"] - ex[key]) < 4 * st["err"], (key, st, ex[key])


def test_mh_refusals(ctx):
    from paper_1912_03278_amd import ihmc
    for lat in (ihmc.Lattice((5, 4), beta=0.4, C=4.1), ihmc.Lattice((4, 4), beta=0.4, C=4.1, h=np.zeros(16))):
        with pytest.raises(ihmc.IhmcError):
            ctx.mh_run(lat, 3)
    r = ctx.mh_run(ihmc.Lattice((4, 4), beta=0.4, C=4.1), 0)
    assert r["m"].size == 0 and r["seconds"] == 0.0
