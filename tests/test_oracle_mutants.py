"""The pins are strong enough: each plausible mistake, planted in a copy of
the oracle's C source and compiled on the CPU, fails at least one pin.

The mutants are text substitutions on ``oracle/edge_oracle.c``; each one is
built into a temporary shared library, swapped in for the real one, and the
pin tests of ``test_oracle_pins.py`` are run against it.
"""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "edge_oracle.c")

MUTANTS = {
    "diagonal_for_4nbr": ("FOUR_NEIGHBOURS[4] = {2, 4, 6, 8}", "FOUR_NEIGHBOURS[4] = {2, 4, 6, 7}"),
    "dropped_neighbour": ("for (int i = 0; i < 4; ++i)", "for (int i = 0; i < 3; ++i)"),
    "wrong_direction": ("DY[9] = {0, -1, -1, -1, 0, +1, +1, +1, 0}",
                        "DY[9] = {0, -1, +1, -1, 0, +1, +1, +1, 0}"),
    "white_is_edge": ("if (p == 0) {", "if (p == 1) {"),
    "clause2_bound": ("if (black_8 <= 1)", "if (black_8 <= 2)"),
    "transposed_index": ("return img[y * W + x] != 0;", "return img[x * H + y] != 0;"),
    "border_ignored": ("return border_pixel;\n    return img", "return 1;\n    return img"),
    "inverted_colour": ("return img[y * W + x] != 0;", "return img[y * W + x] == 0;"),
    "invert_ignored": ("(invert ? !edge : edge)", "(edge)"),
    "clause2_strict": ("if (black_8 <= 1)", "if (black_8 < 1)"),
    "planes_swapped": ("DIRECTION_NEIGHBOUR[4] = {4, 8, 2, 6}", "DIRECTION_NEIGHBOUR[4] = {8, 4, 2, 6}"),
    "plane_diagonal": ("DIRECTION_NEIGHBOUR[4] = {4, 8, 2, 6}", "DIRECTION_NEIGHBOUR[4] = {4, 8, 1, 6}"),
    "plane_no_mask": ("const int mask = 1 - pixel(", "const int mask = 1 | pixel("),
    "threshold_strict": ("grey[i] >= threshold ? 1 : 0", "grey[i] > threshold ? 1 : 0"),
    "threshold_inverted": ("grey[i] >= threshold ? 1 : 0", "grey[i] >= threshold ? 0 : 1"),
    "peel_once_only": ("for (int t = 0; t < iterations; ++t)",
                       "for (int t = 0; t < (iterations > 0); ++t)"),
    "peel_one_extra": ("for (int t = 0; t < iterations; ++t)",
                       "for (int t = 0; t <= iterations; ++t)"),
    "peel_to_black": ("if (edge[i]) cur[i] = 1;", "if (edge[i]) cur[i] = 0;"),
    "peel_layer_of_input": ("oracle_edge_image(cur, out,", "oracle_edge_image(img, out,"),
}


def _pin_suite(golden_dir):
    """The pin tests, run one after another; returns the first failure."""
    from tests import test_oracle_pins_next as nxt
    checks = [
        lambda: nxt.test_fig2_names_match_planes(golden_dir),
        lambda: nxt.test_single_white_neighbour_fires_one_plane(golden_dir),
        lambda: [nxt.test_planes_match_shifted_ands_and_or_to_edge(s, b)
                 for s in [(17, 33)] for b in pins.BORDERS],
        lambda: nxt.test_threshold_by_histogram_and_bounds(),
        lambda: nxt.test_peel_rectangle_closed_form(),
        lambda: [nxt.test_peel_by_taxicab_distance(s, b, q) for s in [(9, 9), (24, 37)]
                 for b in pins.BORDERS for q in (0.5, 0.9)],
        lambda: pins.test_fig1_four_neighbours_are_2_4_6_8(golden_dir),
        lambda: pins.test_fig2_patterns_are_edge_points(golden_dir),
        lambda: pins.test_fig2_patterns_cover_every_edge_point(golden_dir),
        lambda: [pins.test_matches_textbook_morphology(s, b, q)
                 for s in [(17, 33), (1, 7), (7, 1)] for b in pins.BORDERS for q in (0.1, 0.5)],
        lambda: [pins.test_exhaustive_tiny_images(s) for s in [(3, 3), (2, 5), (1, 4)]],
        lambda: [pins.test_closed_forms_whole_image(h, w) for h, w in [(1, 9), (5, 8)]],
        lambda: pins.test_clause2_closed_forms(),
        lambda: [pins.test_invariants(b) for b in pins.BORDERS],
    ]
    for c in checks:
        try:
            c()
        except AssertionError as e:  # the pin caught the mutant
            return e
    return None


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path, monkeypatch, golden_dir):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation site for {name} not found"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new, 1))
    so = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-shared", "-fPIC", "-o", str(so), str(src)],
                   check=True)
    lib = ctypes.CDLL(str(so))
    real = oracle._load()
    for fn in ("oracle_edge_image", "oracle_edge_stack", "oracle_fundamental_edges",
               "oracle_threshold", "oracle_peel"):
        getattr(lib, fn).argtypes = getattr(real, fn).argtypes
        getattr(lib, fn).restype = ctypes.c_int
    monkeypatch.setattr(oracle, "_lib", lib)
    assert _pin_suite(golden_dir) is not None, f"mutant {name} survived every pin"


def test_unmutated_oracle_passes_suite(golden_dir):
    assert _pin_suite(golden_dir) is None
    assert np.array_equal(oracle.edge(np.zeros((2, 2), np.uint8)), np.ones((2, 2), np.uint8))
