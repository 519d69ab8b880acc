"""NTT_ROCTX: with the library's roctx ranges switched on (no profiler
attached, so the ranges go nowhere), the calls compute exactly what they
compute without them. The switch is read once per process, so the calls run
in a child process."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import numpy as np, torch
import paper_2405_11353_amd as ntt, oracle, seeded_inputs as si
torch.cuda.set_device(0)
moduli = si.ntt_primes(60, 18, 3)
for N in (1 << 12, 1 << 16):
    x = si.poly_batch(31 + N, 2, moduli, N)
    plan = ntt.Plan(N, moduli)
    d = torch.from_numpy(x.view(np.int64)).cuda()
    plan.forward(d)
    got = d.cpu().numpy().view(np.uint64).reshape(x.shape)
    assert (got == oracle.ntt_forward_batch(x, moduli)[0]).all(), N
    plan.pointwise_inverse(d[:1], d[1:], d[:1], batch=1)
    c = torch.zeros_like(d[:1])
    a = torch.from_numpy(x.view(np.int64)).cuda()
    plan.polymul(a[:1], a[1:], c, batch=1)
    torch.cuda.synchronize()
    assert torch.equal(c, d[:1]), N
    plan.close()
print("ok", flush=True)
"""


def test_ranges_on_change_nothing():
    env = dict(os.environ, NTT_ROCTX="1", PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    print("case roctx ranges on: child process, N = 2^12 and 2^16", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), (r.stdout + r.stderr)[-4000:]
