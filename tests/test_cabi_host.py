"""CPU checks of the C-ABI library: it loads, exports every symbol the header
declares, and its host-only helpers (Chebyshev roots, schedule merge) agree with
the oracle and with the paper's worked example.  No GPU call is made."""
import json
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from oracle import chebyshev, schedule

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfmp.h")
GOLD = os.path.join(ROOT, "tests", "golden")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pfmp_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1609_02652_amd import pfmp
    lib = pfmp.load()
    syms = declared_symbols()
    assert len(syms) >= 30
    missing = [s for s in syms if not hasattr(lib, s)]
    assert not missing, missing


def test_library_chebyshev_matches_oracle():
    from paper_1609_02652_amd import pfmp
    for n in (4, 10, 16, 32, 64):
        z, a = pfmp.chebyshev(n, 1.2, 0.9)
        zo = chebyshev.roots(n, 1.2, 0.9)
        ao = chebyshev.norm(n, 1.2, 0.9)
        assert max(abs(p - q) for p, q in zip(z, zo)) < 1e-14
        assert abs(a - ao) < 1e-13 * abs(ao)


def test_library_schedule_worked_example():
    """App. B demonstration in ticks of h/6: the library merge equals the paper's T', S'."""
    from paper_1609_02652_amd import pfmp
    g = json.load(open(os.path.join(GOLD, "schedule_demo.json")))
    lam = schedule.OMELYAN_LAMBDA

    def val(s):
        return {"lam": lam, "1-2lam": 1 - 2 * lam}.get(s, None) if s in ("lam", "1-2lam") else float(Fraction(s))

    ticks = lambda l: [int(Fraction(s) * 6) for s in l]
    T, S = pfmp.schedule_build([ticks(g["inputs"]["T1"]), ticks(g["inputs"]["T2"])],
                               [[val(s) for s in g["inputs"]["S1"]], [val(s) for s in g["inputs"]["S2"]]])
    assert T == ticks(g["expected"]["T"])
    assert S[0] == [val(s) for s in g["expected"]["S1"]]
    assert S[1] == [val(s) for s in g["expected"]["S2"]]


@pytest.mark.parametrize("steps", [(10, 20, 40, 80), (10, 15, 40, 120), (3, 7, 11, 13)])
def test_library_schedule_matches_oracle(steps):
    from paper_1609_02652_amd import pfmp
    Ts, Ss = zip(*[schedule.omelyan_2mn(n) for n in steps])
    T, S = schedule.merge(Ts, Ss)
    L = int(np.lcm.reduce([2 * n for n in steps]))
    Ti = [[int(t * L) for t in Tl] for Tl in Ts]
    T2, S2 = pfmp.schedule_build(Ti, [list(s) for s in Ss])
    assert [Fraction(t, L) for t in T2] == T
    for a, b in zip(S, S2):
        assert a == b


def test_library_schedule_rejects_bad_input():
    from paper_1609_02652_amd import pfmp
    with pytest.raises(pfmp.PfmpError):
        pfmp.schedule_build([[0, 2, 2], [0, 3]], [[1, 1, 1], [1, 1]])   # unequal totals


def test_product_path_has_no_cpu_fallback():
    """The binding refuses to run without a GPU instead of falling back."""
    import torch
    from paper_1609_02652_amd import pfmp
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        pfmp.Lattice((4, 4, 4, 4))


def test_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1609_02652_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "pfmp_oracle" not in text and "liboracle" not in text, f
