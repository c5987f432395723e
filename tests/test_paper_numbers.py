"""The precision constants against the numbers the paper prints
(tests/golden/paper_precision_numbers.txt, each line citing its section).

The fixture's numbers are checked for consistency with each other and with
IEEE arithmetic (float32 and float16 spacings), and the precision
experiment's constants and bound are checked against them.  The paper's
measured experiment values are quoted only: its scene is not available, so
they are parity unpinned; the test checks just that they lie under the
paper's own bound.
"""
import math
import os

import numpy as np

import precision_experiment as precision

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "paper_precision_numbers.txt")


def _value(text):
    text = text.strip()
    if "/" in text:
        a, b = text.split("/")
        return float(a) / float(b)
    if "^" in text:
        a, _, p = text.partition("*2^") if "*2^" in text else ("1", "", text.split("^")[1])
        return float(a) * 2.0 ** int(p)
    return float(text)


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                out[k.strip()] = _value(v)
    return out


def test_fixture_parses_every_entry():
    g = _golden()
    assert g["single_eps"] == 2.0 ** -23 and g["half_eps"] == 2.0 ** -10
    assert g["cell_resolution"] == 2.0 ** -24
    assert len(g) == 10


def test_cell_resolution_is_the_float_spacing_at_half():
    g = _golden()
    # the float spacing at 0.5, the largest coordinate magnitude in a cell,
    # is half the machine epsilon: 2^-24 in single, 2^-11 in half precision
    assert float(np.spacing(np.float32(0.5))) == g["cell_resolution"]
    assert float(np.spacing(np.float32(0.5))) == 0.5 * g["single_eps"]
    assert float(np.spacing(np.float16(0.5))) == 0.5 * g["half_eps"]


def test_printed_bounds_are_consistent():
    g = _golden()
    # each step rounds ops_per_step times a coordinate of magnitude <= 0.5
    assert g["step_bound"] == 0.5 * g["ops_per_step"]
    # summing step_bound eps over cell widths that total at most sum_of_widths L
    assert g["length_bound"] == g["step_bound"] * g["sum_of_widths"]
    assert g["angle_bound_scale"] == math.sqrt(2.0)


def test_precision_module_constants_and_bound():
    g = _golden()
    assert precision.EPS32 == g["single_eps"]
    assert precision.EPS16 == g["half_eps"]
    for eps in (g["single_eps"], g["half_eps"]):
        want = math.degrees(math.asin(g["angle_bound_scale"] * g["length_bound"] * eps))
        assert precision.paper_bound_deg(eps) == want


def test_quoted_experiment_lies_under_the_printed_bound():
    g = _golden()
    assert g["quoted_max_angle_deg"] < precision.paper_bound_deg(g["single_eps"])
    assert g["quoted_start_error"] > 0.0
