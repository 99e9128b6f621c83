"""The bench's algorithmic bytes per lattice update (the roofline
denominator) against the per-node count written out for every storage form,
model and lattice: each stored population read once and written once, the
D3Q7 rest population (weight 0) not stored except for the CH-type phase
fields, (phi u) read and written by CH and the Liang models, the nonlocal
model's extra read of h for its multiplier; plus the adjoint's figure."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    return b


# (lattice, model, precision) -> 2 (Qg sg + Qh_stored sh) + extra, by hand
CASES = [
    ("D3Q19_D3Q7", "AC", "mixed_fp16", 2 * (19 * 2 + 6 * 4)),            # 124
    ("D3Q19_D3Q7", "AC", "mixed_bf16", 2 * (19 * 2 + 6 * 4)),            # 124
    ("D3Q19_D3Q7", "AC", "fp32", 2 * (19 * 4 + 6 * 4)),                  # 200
    ("D3Q19_D3Q7", "AC", "fp64", 2 * (19 * 8 + 6 * 8)),                  # 400
    ("D3Q19_D3Q7", "CH", "mixed_fp16", 2 * (19 * 2 + 7 * 4) + 2 * 3 * 4),  # 156
    ("D3Q19_D3Q7", "NL", "mixed_fp16", 2 * (19 * 2 + 6 * 4) + 6 * 4),    # 148
    ("D3Q19_D3Q7", "L18", "mixed_fp16", 2 * (19 * 2 + 6 * 4) + 2 * 3 * 4),  # 148
    ("D3Q19_D3Q7", "L14", "mixed_fp16", 2 * (19 * 2 + 7 * 4) + 2 * 3 * 4),  # 156
    ("D3Q27_D3Q7", "AC", "mixed_fp16", 2 * (27 * 2 + 6 * 4)),            # 156
    ("D3Q27_D3Q7", "AC", "fp64", 2 * (27 * 8 + 6 * 8)),                  # 528
    ("D2Q9_D2Q5", "AC", "fp64", 2 * (9 * 8 + 5 * 8)),                    # 224
]


@pytest.mark.parametrize("lattice,model,precision,expected", CASES)
def test_bytes_per_update(lattice, model, precision, expected):
    b = _bench()
    assert b.bytes_per_update({"lattice": lattice, "model": model}, precision) == expected


def test_adjoint_bytes():
    # lambda in and out (2 x 26 x 8), forward state (26 x 8), 6 workspace values
    # written and read (2 x 6 x 8)
    assert _bench().ADJ_BYTES == 2 * 26 * 8 + 26 * 8 + 2 * 6 * 8 == 720


def test_adjoint_bytes_per_model_and_precision():
    b = _bench()
    # (phi u) in the state, lambda in and out: 3 x 3 x 8 more
    assert b.adjoint_bytes("CH") == b.adjoint_bytes("L18") == 720 + 72
    # the nonlocal model's sum h and dL/dR, written and read: 2 x 2 x 8
    assert b.adjoint_bytes("NL") == 720 + 32
    # Liang2014: (phi u) and mu_phi, lap phi and their adjoints: 72 + 2 x 4 x 8
    assert b.adjoint_bytes("L14") == 720 + 72 + 64
    # float32: every array halved but the float64 phase field (written and read)
    assert b.adjoint_bytes("AC", "fp32") == 26 * 4 + 2 * 26 * 4 + 2 * (8 + 5 * 4) == 368
    assert b.adjoint_bytes("CH", "fp32") == 368 + 3 * 3 * 4 == 404


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, _bench().__file__, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""

