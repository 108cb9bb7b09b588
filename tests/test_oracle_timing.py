"""The all-core oracle timing program (oracle.timing) runs as a child program
on a small case and reports every block once."""
import json
import os
import subprocess
import sys

import numpy as np

import oracle
from synth import random_field

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_all_core_timing_runs_every_block(tmp_path):
    c = np.zeros((2, 2, 2, 3))
    o = oracle.OraclePlan(-21.7e-24, 128e9, 40.0, 2, 0.3, 2, 512, 128, c)
    x = random_field((2, 3000), 5, power_w=1e-3)
    case = tmp_path / "case.npz"
    np.savez(case, x=x, coeffs=c, beta2_s2_km=o.beta2_s2_km, sample_rate=o.sample_rate, step_km=o.step_km,
             n_steps=o.n_steps, rho=o.rho, n_sb=o.n_sb, n_block=o.n_block, n_overlap=o.n_overlap)
    res = subprocess.run([sys.executable, "-m", "oracle.timing", str(case), "3"], cwd=ROOT, capture_output=True,
                         text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    t = json.loads(res.stdout.strip().splitlines()[-1])
    assert t["blocks"] == o.n_blocks(3000) and t["workers"] == 3 and t["wall_s"] > 0
