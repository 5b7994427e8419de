"""The oracle's pins catch planted mistakes. Each case copies oracle.c, plants
one plausible error (a boundary rule, a dropped edge, a flipped orientation, a
wrong vertex in a difference, a box that is not half-open, the wrong
tie-break, a miscounted unit of work, a miscounted or mis-joined block),
builds the copy with gcc on the CPU, points the oracle module at it, and checks that at least one pin of test_oracle_pins fails. Nothing here
touches a GPU or the mapping library."""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("straddle_counts_the_upper_end",
     "int a_above = ay > py, b_above = by > py;",
     "int a_above = ay >= py, b_above = by >= py;"),
    ("crossing_not_strictly_right",
     "return (by > ay) ? (lhs < rhs) : (lhs > rhs);",
     "return (by > ay) ? (lhs <= rhs) : (lhs >= rhs);"),
    ("orientation_flipped",
     "return (by > ay) ? (lhs < rhs) : (lhs > rhs);",
     "return (by < ay) ? (lhs < rhs) : (lhs > rhs);"),
    ("wrong_vertex_in_a_difference",
     "i128 lhs = (i128)(px - ax) * (i128)(by - ay);",
     "i128 lhs = (i128)(px - bx) * (i128)(by - ay);"),
    ("closing_edge_dropped",
     "for (int64_t k = 0; k < m; ++k) {\n    int64_t k1",
     "for (int64_t k = 0; k + 1 < m; ++k) {\n    int64_t k1"),
    ("box_open_at_its_low_corner",
     "return bx[0] <= px && px < bx[1] && bx[2] <= py && py < bx[3];",
     "return bx[0] < px && px < bx[1] && bx[2] < py && py < bx[3];"),
    ("largest_id_wins",
     "if (best < 0 || b < best) best = (int32_t)b;",
     "if (best < 0 || b > best) best = (int32_t)b;"),
    ("last_hit_wins_in_brute_force",
     "        if (best < 0) best = (int32_t)b;",
     "        best = (int32_t)b;"),
    # the work counters that price the method per point
    ("box_tests_counted_for_survivors_only",
     "c.bbox_tests++;\n            if (in_box(h->box[l + 1] + 4 * e, px, py)) vpush(&nxt, e);",
     "if (in_box(h->box[l + 1] + 4 * e, px, py)) { c.bbox_tests++; vpush(&nxt, e); }"),
    ("top_level_box_tests_not_counted",
     "c.bbox_tests++;\n        if (in_box(h->box[0] + 4 * g, px, py)) vpush(&cur, g);",
     "if (in_box(h->box[0] + 4 * g, px, py)) vpush(&cur, g);"),
    ("x_range_closed_at_its_top",
     "if (lo <= px && px < hi) c.x_ambiguous++;",
     "if (lo <= px && px <= hi) c.x_ambiguous++;"),
    ("straddle_count_owns_the_upper_end",
     "if ((ay > py) != (by > py)) {\n            c.straddles++;",
     "if ((ay >= py) != (by >= py)) {\n            c.straddles++;"),
    ("closing_edge_not_counted",
     "c.edge_tests += m;",
     "c.edge_tests += m - 1;"),
    ("candidates_counted_once_per_point",
     "c.leaf_cands++;",
     "c.leaf_cands += (t == 0);"),
    # per-block aggregation
    ("out_of_range_ids_not_counted",
     "    else counts[nb]++;",
     "    else if (b == -1) counts[nb]++;"),
    ("join_misses_the_last_block",
     "out[i] = (b >= 0 && b < nb) ? table[b] : fill;",
     "out[i] = (b >= 0 && b < nb - 1) ? table[b] : fill;"),
]


def _pin_calls():
    calls = [("hand_cases_golden", pins.test_hand_cases_golden, ())]
    calls += [("rectangle %s" % (r,), pins.test_rectangle_closed_form, (r,)) for r in pins.RECTS]
    calls += [("rectilinear %s" % n, pins.test_rectilinear_closed_form, (n,)) for n in sorted(pins.RECTILINEAR)]
    calls += [("rational %s" % n, pins.test_exact_rational_reference, (n,)) for n in sorted(pins.NONRECT)]
    calls += [("random stars", pins.test_random_star_polygons_rational_and_winding, ()),
              ("box conservative", pins.test_box_is_conservative, ()),
              ("unjittered grid", pins.test_unjittered_grid_closed_form, ()),
              ("partition grid1k", pins.test_partition_invariant, ("grid1k",)),
              ("overlapping rectangles", pins.test_overlapping_rectangles_smallest_id, ()),
              ("hierarchy == brute grid1k", pins.test_hier_equals_brute_grid1k, ()),
              ("work counters", pins.test_hierarchy_work_counts_closed_form, ()),
              ("count and join", pins.test_count_and_join_per_block_closed_form, ())]
    return calls


@pytest.mark.parametrize("name, old, new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, monkeypatch, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "the planted text must occur once"
    mutant = tmp_path / "oracle_mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", str(mutant), "-o", str(lib)])
    monkeypatch.setattr(oracle, "_LIB_PATH", str(lib))
    monkeypatch.setattr(oracle, "_lib", None)
    caught = []
    for label, fn, args in _pin_calls():
        try:
            fn(*args)
        except AssertionError:
            caught.append(label)
    monkeypatch.setattr(oracle, "_lib", None)  # the next use reloads the real oracle
    assert caught, "no pin caught the planted mistake " + name


def test_unmutated_copy_passes_every_pin(tmp_path, monkeypatch):
    """The same procedure on an unmodified copy: every pin passes, so a caught
    mutant is caught because of its mistake."""
    lib = tmp_path / "liboracle_copy.so"
    subprocess.check_call(["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", SRC, "-o", str(lib)])
    monkeypatch.setattr(oracle, "_LIB_PATH", str(lib))
    monkeypatch.setattr(oracle, "_lib", None)
    for label, fn, args in _pin_calls():
        fn(*args)
    monkeypatch.setattr(oracle, "_lib", None)
