"""Host-side parts of the benchmark.  Its check that an interleaved-field run
ends on the split run's state compares 64-bit digests of the pools' valid
records: the digest must change with any bit of a valid record or their
order, and not with anything outside the valid records (host tensors stand
in for device ones).  It measures one GPU and refuses more."""
import importlib.util
import os
import types

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _pool(vdt):
    g = torch.Generator().manual_seed(5)
    base = torch.tensor([0, 10, 25], dtype=torch.int64)
    cap = torch.tensor([10, 15, 5], dtype=torch.int64)
    count = torch.tensor([3, 15, 0], dtype=torch.int64)
    return types.SimpleNamespace(
        x=torch.randn(3, 30, dtype=torch.float64, generator=g),
        v=torch.randn(3, 30, generator=g).to(vdt), tau=torch.rand(30, generator=g).to(vdt),
        id=torch.arange(30, dtype=torch.int64), base=base, cap=cap, count=count)


def test_digest_sees_valid_records_only():
    b = _bench()
    for vdt in (torch.float64, torch.float32):
        p = _pool(vdt)
        d0 = b.state_digest(p)
        assert d0 == b.state_digest(_pool(vdt))
        # one ulp in a valid position, a valid velocity, a valid id
        for name, idx in (("x", (1, 12)), ("v", (2, 0)), ("tau", (24,)), ("id", (11,))):
            q = _pool(vdt)
            t = getattr(q, name)
            if t.is_floating_point():
                t[idx] = torch.nextafter(t[idx], torch.tensor(float("inf"), dtype=t.dtype))
            else:
                t[idx] += 1
            assert b.state_digest(q) != d0, name
        # two valid records swapped
        q = _pool(vdt)
        q.x[:, [11, 12]] = q.x[:, [12, 11]]
        assert b.state_digest(q) != d0
        # slots past a count (segment 0 holds 3 of 10; segment 2 none)
        q = _pool(vdt)
        q.x[:, 5] = 7.0
        q.v[:, 27] = 1.0
        q.id[29] = -1
        assert b.state_digest(q) == d0


def test_more_than_one_gpu_is_refused_with_a_message():
    """bench.py measures one GPU; --gpus above 1 exits before touching a
    device, with a message that says so."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""
