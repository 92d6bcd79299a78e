"""Planted mistakes: each plausible slip in the oracle's arithmetic must fail some pin.

A mutated copy of the oracle's C source is compiled into a temporary directory (the committed
oracle is untouched), swapped in for the duration of the check, and the pin battery of
``test_oracle_pins`` is run against it; at least one pin must fail.
"""

import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as O
import oracle.build as OB

from . import test_oracle_pins as P

MUTATIONS = {
    "gain_sign": ("i128 g = (i128)W * (i128)acc[c] - Ki * (i128)Sig[c];",
                  "i128 g = (i128)W * (i128)acc[c] + Ki * (i128)Sig[c];"),
    "stay_drops_own_degree": ("r.stay = (i128)W * kd - Ki * ((i128)Sig[d] - Ki);",
                              "r.stay = (i128)W * kd - Ki * ((i128)Sig[d]);"),
    "tie_to_largest": ("(g == r.best_gain && c < r.best)", "(g == r.best_gain && c > r.best)"),
    "swap_rule_direction": ("csize[r.best] == 1 && r.best > d", "csize[r.best] == 1 && r.best < d"),
    "non_strict_move": ("if (r.best >= 0 && r.best_gain > r.stay)",
                        "if (r.best >= 0 && r.best_gain >= r.stay)"),
    "self_loop_is_candidate": ("if (j == i) continue; /* self-loop", "if (0) continue; /* self-loop"),
    "modularity_wrong_index": ("if (C[idx[e]] == C[i]) sigma += w[e];",
                               "if (idx[e] == C[i]) sigma += w[e];"),
    "modularity_drops_square": ("sq += (u128)Sig[c] * Sig[c];", "sq += (u128)Sig[c];"),
    "aggregate_transposed": ("int32_t b = map[idx[e]];", "int32_t b = map[i];"),
    "threshold_off_by_two": ("u128 div = 2;", "u128 div = 1;"),
    "sync_reads_current_state": ("Cn[i] = r.target;", "Cn[i] = r.target; C[i] = r.target;"),
    "class_hash_constant": ("z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;",
                            "z = (z ^ (z >> 27)) * 0x94D049BB133111EAull;"),
    "step_moves_unlisted": ("int64_t i = verts ? verts[t] : t;\n      decision",
                            "int64_t i = verts ? (verts[t] + 1) % n : t;\n      decision"),
    "async_no_sigma_update": ("Sig[c] += K[i];\n      csize[d] -= 1;", "csize[d] -= 1;"),
    "level_records_pass_map": ("memcpy(levels + (size_t)(*n_levels) * (size_t)n, top,",
                               "memcpy(levels + (size_t)(*n_levels) * (size_t)n, map,"),
    "prep_reverses_loops": ("if ((flags & ORC_PREP_SYM) && src[e] != dst[e]) {",
                            "if ((flags & ORC_PREP_SYM)) {"),
    "prep_max_sums": ("if (flags & ORC_PREP_MAX) {\n        if (a[i].w > wout[nnz - 1])",
                      "if (0) {\n        if (a[i].w > wout[nnz - 1])"),
    "prep_merges_across_rows": ("idx[nnz - 1] == a[i].v && i > 0 && a[i - 1].u == a[i].u",
                                "idx[nnz - 1] == a[i].v"),
    "prep_loop_weight_two": ("a[k].v = (int32_t)v; a[k].w = 1; k++;",
                             "a[k].v = (int32_t)v; a[k].w = 2; k++;"),
    "colour_ascending_priority": ("if (x->prio != y->prio) return x->prio > y->prio ? -1 : 1;",
                                  "if (x->prio != y->prio) return x->prio < y->prio ? -1 : 1;"),
    "colour_leftover_reuses_last": ("    int32_t c = K - 1;\n    for (int32_t k = 0; k < K - 1; k++)",
                                    "    int32_t c = K - 2;\n    for (int32_t k = 0; k < K - 1; k++)"),
    "colour_mask_shifted": ("used |= 1u << colour[u];", "used |= 2u << colour[u];"),
    "partition_labels_not_offset": ("for (int64_t v = v0; v < v1; v++) label[v] += (int32_t)next_label;",
                                    "for (int64_t v = v0; v < v1; v++) label[v] += 0;"),
    "partition_merge_skipped": ("for (int64_t v = 0; v < n; v++) top[v] = stop[map[v]];",
                                "for (int64_t v = 0; v < n; v++) top[v] = map[v];"),
    "partition_keeps_part_edge": ("if (idx[e] >= v0 && idx[e] < v1) {",
                                  "if (idx[e] >= v0 && idx[e] < v1 && idx[e] != v1 - 1) {"),
    "class_pass_index": (": colour_classes ? colour[v] : orc_vertex_class(p, substeps, v);",
                         ": colour_classes ? colour[v] : orc_vertex_class(0, substeps, v);"),
    "pass_keeps_non_increasing": ("if (!(q_after > q_before)) break;",
                                  "if (q_after == q_before) break;"),
    "gain_product_wraps_64": ("i128 g = (i128)W * (i128)acc[c] - Ki * (i128)Sig[c];",
                              "i128 g = (i128)(W * acc[c]) - Ki * (i128)Sig[c];"),
    "modularity_product_wraps_64": ("i128 q = (i128)((u128)W * sigma) - (i128)sq;",
                                    "i128 q = (i128)(W * sigma) - (i128)sq;"),
    "level_cap_off_by_one": ("if (levels && n_levels && *n_levels < max_levels) {",
                             "if (levels && n_levels && *n_levels + 1 < max_levels) {"),
}


def battery():
    """The pins, run against whatever library ``oracle.lib()`` returns."""
    P.test_threshold_values()
    for W in [14, 10**6 + 3, 2**62]:
        P.test_threshold_is_exact_floor(W)
    P.test_modularity_closed_form_values()
    P.test_modularity_all_in_one_and_singletons()
    P.test_modularity_matches_pairwise_definition_with_self_loops()
    P.test_single_move_identity()
    P.test_sync_iteration_bruteforce()
    P.test_sync_zero_gain_move_not_taken()
    P.test_vertex_class_matches_splitmix64()
    P.test_sync_step_on_a_subset_bruteforce()
    P.test_async_exact_change_per_iteration()
    P.test_aggregation_invariants()
    P.test_worked_example_two_triangles()
    P.test_single_edge_run()
    P.test_ring_of_cliques_recovered()
    P.test_levels_ring_of_k4_hand_derived()
    P.test_levels_edge_cases()
    P.test_pass_that_lowers_modularity_is_dropped()
    P.test_run_classes_are_the_hashed_classes()
    P.test_big_weights_modularity_and_single_moves()
    P.test_big_weights_sync_async_aggregation()
    from . import test_oracle_colour as PC
    for K in (2, 8, 32):
        PC.test_matches_jones_plassmann_rounds(K)
        PC.test_shortcut_rounds_equal_sequential_first_fit(K)
    from . import test_oracle_partition as PT
    PT.test_two_triangles_hand_derived()
    PT.test_components_as_parts(8)
    PT.test_matches_composition(4)
    from . import test_oracle_prepare as PP
    PP.test_golden_small()
    for f in PP.FLAG_SETS:
        PP.test_matches_dense_definition(f)


def test_battery_passes_on_committed_oracle():
    battery()


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name):
    old, new = MUTATIONS[name]
    src = open(OB.SRC).read()
    assert src.count(old) == 1, name
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "mut.c")
        lib = os.path.join(d, "libmut.so")
        open(path, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-std=gnu11", "-O1", "-fopenmp", "-fPIC", "-shared",
                               "-w", "-o", lib, path])
        O.lib()  # make sure the real one is loaded first
        saved = O._LIB
        O._LIB = ctypes.CDLL(lib)
        try:
            with pytest.raises(AssertionError):
                battery()
        finally:
            O._LIB = saved
