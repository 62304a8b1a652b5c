"""FEWHA_TRACE=1 (roctx ranges around the library's calls and the solve's phases) changes no
result: a traced frame chain in a child process equals, bitwise, the same chain untraced."""
import os
import subprocess
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHAIN = """
import sys
sys.path.insert(0, %r)
import numpy as np, torch
from paper_2009_00946_amd import fewha, synth
cfg = synth.load_config("t1_mixed")
P = fewha.Plan(cfg, precision="fp32")
c, a = P.zeros(P.n_coef), P.zeros(P.n_act)
for f in range(3):
    phi = torch.as_tensor(synth.layer_screens_flat(cfg, f), dtype=P.dtype, device=P.device)
    s = P.apply_A(P.dwt_forward(phi))
    P.reconstruct(s, c, cfg["n_iter"], a_prev=a, gain=0.5, out=a, warm=f > 0, refresh=f == 2)
torch.cuda.synchronize()
assert P.last_status() == 0
np.save(sys.argv[1], np.concatenate([c.double().cpu().numpy(), a.double().cpu().numpy()]))
""" % ROOT


def _run(path, trace):
    env = dict(os.environ)
    env.pop("FEWHA_TRACE", None)
    if trace:
        env["FEWHA_TRACE"] = "1"
    r = subprocess.run([sys.executable, "-c", CHAIN, path], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return np.load(path)


def test_traced_chain_equals_untraced(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print("\n[trace] t1_mixed fp32 chain, traced and untraced", flush=True)
    a = _run(str(tmp_path / "plain.npy"), False)
    b = _run(str(tmp_path / "traced.npy"), True)
    assert np.array_equal(a, b)
