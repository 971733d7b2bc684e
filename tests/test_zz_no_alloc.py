"""psms_cheb_helmholtz_noalloc (the library's own device scratch, no workspace)
against psms_cheb_helmholtz (caller workspace) through the C ABI: the same kernel
on the same inputs, so the results must be identical, and close to the dense
FP64 oracle.  Two calls in a row, the second smaller, so that the second runs on
scratch that still holds the first call's values."""
import math

import numpy as np
import pytest

from oracle import channel as ch

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BETA_NS = 2.0 * 150.0 / 1e-4


def _lines(nc, nl, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((nc + 1, nl)) + 1j * rng.standard_normal((nc + 1, nl))
    return x * np.exp(-0.03 * np.arange(nc + 1))[:, None]


@pytest.mark.parametrize("kind", ["dirichlet", "neumann"])
def test_noalloc_helmholtz_equals_the_workspace_call(kind):
    from paper_2406_01322_amd import psms
    # (nc, lines): the second call is smaller than the first; the first fills most
    # of the 2^20-double scratch (129 * 7310 = 942,990 doubles)
    for call, (nc, nl, seed) in enumerate([(128, 7310, 1), (32, 37, 2)]):
        print("noalloc call %d: nc %d, %d lines, %s" % (call, nc, nl, kind), flush=True)
        rng = np.random.default_rng(seed + 10)
        g = torch.from_numpy(_lines(nc, nl, seed)).cuda()
        beta = torch.from_numpy(BETA_NS * (0.5 + rng.random(nl))).cuda()
        bcv = torch.from_numpy(rng.standard_normal((nl, 2)) + 1j * rng.standard_normal((nl, 2))).cuda()
        want = psms.cheb_helmholtz(g, beta, kind, bcv)
        got = psms.cheb_helmholtz_noalloc(g, beta, kind, bcv)
        torch.cuda.synchronize()
        assert torch.equal(got, want), call
        # and the oracle on a few lines (the dense LU; the conditioning bar of the
        # workspace call's own parity test)
        gh, bh, vh, oh = (t.cpu().numpy() for t in (g, beta, bcv, got))
        for l in (0, nl // 2, nl - 1):
            ref = ch.helmholtz(gh[:, l], bh[l], kind, vh[l, 0], vh[l, 1])
            assert np.max(np.abs(oh[:, l] - ref)) <= 1e-11 * np.max(np.abs(ref)), (call, l)


def test_noalloc_helmholtz_rejects_inputs_beyond_the_scratch():
    from paper_2406_01322_amd import psms
    nc = 128
    limit = (1 << 20) // (nc + 1)
    g = torch.zeros((nc + 1, limit + 1), dtype=torch.complex128, device="cuda")
    beta = torch.ones(limit + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(psms.PsmsError) as e:
        psms.cheb_helmholtz_noalloc(g, beta)
    assert e.value.code == -2
    assert "scratch" in str(e.value)
