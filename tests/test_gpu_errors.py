"""Error paths forced from the host on a GPU: the allocation-failure hook
(FEA_FAIL_ALLOC_AT=n fails the n-th device allocation of the process) must
turn into FEA_ENOMEM from the call that allocates, with no launch left
half-done, and later calls must still work."""
import os
import subprocess
import sys

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = r'''
import sys
sys.path.insert(0, sys.argv[1])
import torch
import meshgen as mg
import paper_1805_03949_amd as fea
m = mg.hybrid_bands(4, seed=2, jitter=0.2)
dm = fea.DeviceMesh(m, device="cuda:0")
codes = []
for attempt in range(2):
    try:
        g = dm.graph()
        v, r, st = dm.assemble(g, variant=fea.ROWSYM)
        torch.cuda.synchronize()
        codes.append(0 if int(st.item()) == -1 else 99)
        g.destroy()
    except fea.FeaError as e:
        codes.append(e.code)
        print("error:", e.msg, flush=True)
print("codes", codes, flush=True)
'''


@pytest.mark.parametrize("n", [1, 4, 12, 30])
def test_injected_allocation_failure_reports_enomem(n):
    env = {**os.environ, "FEA_FAIL_ALLOC_AT": str(n)}
    print(f"[case] FEA_FAIL_ALLOC_AT={n}", flush=True)
    p = subprocess.run([sys.executable, "-c", SCRIPT, ROOT], env=env, stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=300)
    assert p.returncode == 0, p.stdout[-3000:]
    line = [l for l in p.stdout.splitlines() if l.startswith("codes")][-1]
    codes = eval(line.split(" ", 1)[1])
    # the first attempt hits the injected failure (graph build or the first
    # upper-triangle assembly allocate well over 30 buffers); the second runs
    assert codes[0] == -3, p.stdout[-3000:]
    assert "(injected)" in p.stdout
    assert codes[1] == 0, p.stdout[-3000:]
