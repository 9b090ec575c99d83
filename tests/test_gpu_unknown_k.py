"""GPU parity of the unknown-K strategy (Sec. II-G) through the C ABI: the
rung chosen on the device equals the oracle's bottom-up choice, and the
output equals the oracle's run at that M."""
import sys

import numpy as np
import pytest

import oracle
import sftgen

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t

    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def sft():
    import paper_1407_8315_amd as m

    return m


@pytest.mark.parametrize("n,k,L,m_max,dtype", [
    (1 << 14, 100, 4, 4096, "c128"),
    (1 << 12, 3, 4, 1024, "c128"),        # K <= L: solved at d = N
    (1 << 16, 400, 2, 1 << 14, "c128"),
    (1 << 20, 1000, 4, 1 << 14, "c64"),   # the exact workload's size, K not given
    (1 << 12, 600, 4, 64, "c128"),        # every rung flags: the last rung's list
])
def test_unknown_k_matches_oracle(torch, sft, n, k, L, m_max, dtype):
    say(f"[unknown K] n={n} k={k} L={L} m_max={m_max} {dtype}")
    npdt = np.complex128 if dtype == "c128" else np.complex64
    s = sftgen.make_signal(n, k, 600 + k, amp="gauss", dtype=npdt)
    plan = sft.Plan(dict(n=n, k=1, m=m_max, l=L, dtype=dtype, flags=sft.SFT_FLAG_UNKNOWN_K))
    res, m = plan.unknown_k(torch.from_numpy(s.x).cuda(), capacity=m_max * L, stats=True)
    loc, val = res.host()
    plan.close()
    ref, m_ref = oracle.sfft_unknown_k(s.x, n, L, m_max=m_max)   # FP64 FFTs
    say(f"  M chosen {m} (oracle {m_ref}), flagged {res.stats['flagged_bins']}")
    assert m == m_ref
    assert loc.tolist() == ref.locs.tolist()
    assert res.stats["flagged_bins"] == ref.flagged_bins
    if len(loc):
        ref64 = oracle.sfft_exact(s.x, n, m, L)
        common, ia, ib = np.intersect1d(loc, ref64.locs, return_indices=True)
        tol = 1e-10 if dtype == "c128" else 1e-5
        assert np.linalg.norm(val[ia] - ref64.vals[ib]) <= tol * max(1.0, np.linalg.norm(ref64.vals[ib]))
