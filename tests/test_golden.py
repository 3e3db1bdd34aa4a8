"""The paper's printed constants used by the oracle and the library are read from the golden
fixture (each line cites its section), and the defaults of the oracle and
the binding agree with them."""
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def golden():
    vals = {}
    for line in open(os.path.join(ROOT, "tests", "golden", "paper_constants.txt")):
        line = line.split("#", 1)[0].strip()
        if "=" in line:
            k, v = line.split("=", 1)
            vals[k.strip()] = float(v)
    return vals


def test_schwarz_tolerance_defaults_match_paper():
    import oracle
    from paper_2605_09097_amd import binding

    g = golden()
    assert oracle.schwarz_opts(2).eps_conv == g["eps_conv"]
    assert binding.schwarz_opts(2).eps_conv == g["eps_conv"]


def test_speedups_printed():
    g = golden()
    assert (g["speedup_ratio1"], g["speedup_ratio2"], g["speedup_ratio5"]) == (6.61, 9.15, 4.34)
