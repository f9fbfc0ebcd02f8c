"""Debug and tracing switches of the library, each in a child process (they
are read once per process): ITC_DEBUG_VALIDATE rejects non-finite FP32/FP64
weights before anything is enqueued; ITC_TRACE opens roctx ranges and leaves
results unchanged."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

VALIDATE = r"""
import sys, torch
sys.path.insert(0, ROOT)
from paper_1310_7114_amd import itc
x = torch.rand(40, 50, device="cuda")
itc.precompute(x, 2.0)                              # finite: accepted
x[7, 9] = float("nan")
try:
    itc.precompute(x, 2.0)
    print("accepted")
except itc.ItcError as e:
    print("rejected", e.status, "non-finite" in e.detail)
p = itc.BatchPlan([torch.rand(30, 40), torch.rand(20, 24)], [4, 4], [2.0, 2.0], [3, 3])
p.weights[5] = float("inf")
try:
    p.precompute()
    print("accepted")
except itc.ItcError as e:
    print("rejected", e.status, "non-finite" in e.detail)
"""

TRACE = r"""
import sys, torch
sys.path.insert(0, ROOT)
from paper_1310_7114_amd import itc, synth
c = synth.config1_case(1)
m = itc.precompute(torch.from_numpy(c.img).cuda(), c.sigma)
w, tr, done = itc.fit(m, torch.from_numpy(c.w0).cuda(), 10)
torch.cuda.synchronize()
print(repr(w.cpu().double().numpy().tobytes().hex()[:64]), float(tr[-1]))
"""


def run_child(code, **env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-c", code.replace("ROOT", repr(ROOT))], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout.strip().splitlines()


def test_debug_validate_rejects_nonfinite_weights(gpu_lib):
    lines = run_child(VALIDATE, ITC_DEBUG_VALIDATE="1")
    assert lines[-2:] == ["rejected 2 True", "rejected 2 True"], lines


def test_trace_ranges_leave_results_unchanged(gpu_lib):
    plain = run_child(TRACE)
    traced = run_child(TRACE, ITC_TRACE="1")
    assert plain[-1] == traced[-1]
