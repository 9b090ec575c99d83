"""sft_exact_noalloc (static workspace, no device allocation) against
sft_exact, through the C ABI: two calls in a row, the second on a smaller
input, each compared with sft_exact on the same parameters and input
(support identical; values within 1e-5 relative for complex64 input, the
amplitude bar of the exact workload, and 1e-10 for complex128), and the
complex128 case also with the FP64 oracle."""
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


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_noalloc_equals_exact_on_two_calls(torch, sft):
    cases = [
        (dict(n=1 << 20, k=1000, m=4096, l=4, dtype="c64"), np.complex64, "gauss", 1e-5),
        (dict(n=1 << 14, k=50, m=128, l=4, dtype="c128"), np.complex128, "unit", 1e-10),
    ]
    for i, (p, npdt, amp, tol) in enumerate(cases):
        say(f"[noalloc] call {i}: {p}")
        s = sftgen.make_signal(p["n"], p["k"], sftgen.BASE_SEED + 700 + i, amp=amp, dtype=npdt)
        x = torch.from_numpy(s.x).to("cuda")
        plan = sft.Plan(p)
        ref_out = plan.exact(x, stats=True)
        torch.cuda.synchronize()
        l_ref, v_ref = ref_out.host()
        out = plan.new_output(p["m"] * p["l"])
        out.count.fill_(-1)
        out.loc.fill_(-7)
        sft.exact_noalloc(x, p, out)
        torch.cuda.synchronize()
        loc, val = out.host()
        plan.close()
        say(f"  {len(loc)} entries, sft_exact {len(l_ref)}; max rel. value difference "
            f"{rel(val, v_ref) if len(loc) == len(l_ref) and len(loc) else float('nan'):.2e}")
        assert int(out.count.item()) == len(l_ref)
        assert loc.tolist() == l_ref.tolist()
        assert rel(val, v_ref) <= tol
        if npdt == np.complex128:
            ref = oracle.sfft_exact(s.x, p["n"], p["m"], p["l"])
            assert loc.tolist() == ref.locs.tolist() == s.locs.tolist()
            assert rel(val, ref.vals) <= 1e-10


def test_noalloc_capacity_and_reuse_after_a_larger_call(torch, sft):
    """A small capacity keeps the smallest locations and the full count; a
    later call on a larger signal in the same workspace is again exact."""
    p = dict(n=1 << 16, k=200, m=1024, l=4, dtype="c64")
    s = sftgen.make_signal(p["n"], p["k"], 31, amp="unit", dtype=np.complex64)
    x = torch.from_numpy(s.x).to("cuda")
    plan = sft.Plan(p)
    out = plan.new_output(16)
    say("[noalloc] capacity 16")
    sft.exact_noalloc(x, p, out, capacity=16)
    torch.cuda.synchronize()
    assert int(out.count.item()) == p["k"]
    assert out.loc[:16].cpu().numpy().tolist() == s.locs[:16].tolist()
    plan.close()
    q = dict(n=1 << 18, k=2000, m=8192, l=3, dtype="c64")
    s2 = sftgen.make_signal(q["n"], q["k"], 32, amp="unit", dtype=np.complex64)
    x2 = torch.from_numpy(s2.x).to("cuda")
    plan2 = sft.Plan(q)
    ref = plan2.exact(x2).host()
    out2 = plan2.new_output(q["m"] * q["l"])
    say("[noalloc] M = 8192, L = 3")
    sft.exact_noalloc(x2, q, out2)
    torch.cuda.synchronize()
    loc, val = out2.host()
    plan2.close()
    assert loc.tolist() == ref[0].tolist()
    assert rel(val, ref[1]) <= 1e-5
