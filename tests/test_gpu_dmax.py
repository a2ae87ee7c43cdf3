"""findDmax on the device (design space exploration, Algorithm 1's findDmax; the noise
study) against the oracle's trials: every trial's D_i must be equal, for BFV, rounded BFV
and BGV, one and two limbs, 30- and 24-bit primes, trials that fail at the first term, in
the middle and never (D_i = d_cap)."""
import numpy as np
import pytest

import paper_2511_00737_amd as ep
from oracle import dmax
from oracle.params import Params as OParams, default_primes

from gpu_helpers import torch_cuda

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("scheme,t,L,bits,d_cap,K,qbits,cbits", [
    ("bfv", 786433, 2, 30, 24, 2, 1, 8),
    ("bfv", 40961, 2, 24, 40, 2, 1, 8),
    ("bgv", 786433, 2, 24, 40, 2, 1, 8),
    ("bfv-r", 786433, 2, 24, 40, 3, 2, 4),
    ("bgv", 65537, 2, 30, 12, 2, 1, 8),
    ("bgv", 12289, 1, 30, 16, 2, 1, 8),
])
def test_find_dmax_matches_oracle_trials(scheme, t, L, bits, d_cap, K, qbits, cbits):
    torch_cuda()
    N = 2048
    q = tuple(default_primes(N, L, bound=1 << bits))
    o = OParams(N=N, q=q, t=t, D=d_cap, K=K, F=8, scheme=scheme, qbits=qbits)
    o.validate()
    e = ep.Params(N=N, q=q, t=t, D=d_cap, K=K, F=16, scheme=scheme, qbits=qbits)
    seed, trials = 5, 3
    got = ep.ephdc_find_dmax(e, seed, trials, d_cap, cbits)
    want = [dmax.trial(o, seed + i, d_cap, cbits) for i in range(trials)]
    assert got.tolist() == want


def test_find_dmax_rejects_what_it_does_not_implement():
    torch_cuda()
    q = tuple(default_primes(2048, 3))
    with pytest.raises(ep.EphdcError) as ei:
        ep.ephdc_find_dmax(ep.Params(N=2048, q=q, t=65537, D=8, K=2, F=16), 1, 1, 8)
    assert ei.value.status == ep.ERR_UNSUPPORTED  # three limbs
    with pytest.raises(ep.EphdcError) as ei:
        ep.ephdc_find_dmax(ep.Params(N=2048, q=q[:2], t=65537, D=8, K=2, F=16), 1, 1, 8, cbits=9)
    assert ei.value.status == ep.ERR_ARG
