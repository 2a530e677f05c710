"""Planted mistakes in the CPU oracle must be caught by its pins.

Each mutant is a copy of the oracle source with one plausible slip (a
flipped comparison, a dropped term, a transposed operand, an off-by-one),
compiled on the CPU. The pin tests of ``test_oracle_pins`` -- excluding the
cross-check against the second transcription -- run against it, and at least
one must fail. This shows the pins constrain every step of the oracle.
"""
import os
import subprocess
import tempfile

import pytest

from oracle import oracle as O
from tests import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(O.__file__), "jet_oracle.c")

# (name, exact source text, replacement)
MUTANTS = [
    ("argmax tie to larger part", "(conn[p] == bestc && p < best)) { best = p; bestc = conn[p]; }\n        }\n        conn_s",
     "(conn[p] == bestc && p > best)) { best = p; bestc = conn[p]; }\n        }\n        conn_s"),
    ("filter not strict", "-F[v] < thr", "-F[v] <= thr"),
    ("filter ratio transposed", "((int64_t)cn * conn[ps]) / cd", "((int64_t)cd * conn[ps]) / cn"),
    ("ord by smaller gain", "(F[u] > F[v] || (F[u] == F[v] && u < v))", "(F[u] < F[v] || (F[u] == F[v] && u < v))"),
    ("ord tie by larger id", "(F[u] > F[v] || (F[u] == F[v] && u < v))", "(F[u] > F[v] || (F[u] == F[v] && u > v))"),
    ("afterburner sign", "else if (q == P[v]) f2 -= g->adjwgt[e];", "else if (q == P[v]) f2 += g->adjwgt[e];"),
    ("afterburner drops zero gain", "if (f2 >= 0) { move[v] = 1; nM++; }", "if (f2 > 0) { move[v] = 1; nM++; }"),
    ("afterburner ignores ord", "q = pd[u];\n", ";\n"),
    ("slot off by one", "return 2 + fl;", "return 1 + fl;"),
    ("inclusive eviction test", "if (s >= need) break;", "if (s + g->vwgt[L[i].v] >= need) break;"),
    ("eligibility factor", "3 * ((int64_t)k * w[ps] - W)", "2 * ((int64_t)k * w[ps] - W)"),
    ("strong loss uses sum", "int64_t mean = cnt ? sum / cnt : 0;", "int64_t mean = sum;"),
    ("weak loss sign", "loss[v] = conn[ps] - conn[best];", "loss[v] = conn[best] - conn[ps];"),
    ("cut double counted", "if (u > v && P[u] != P[v]) c += g->adjwgt[e];", "if (P[u] != P[v]) c += g->adjwgt[e];"),
    ("locks ignored", "if (locked[v]) continue;", ""),
    ("limit lambda sign", "(1000000 + (__int128)lambda_ppm)", "(1000000 - (__int128)lambda_ppm)"),
    ("no deadzone", "if (slack < div) return o - 1;\n    return o - slack / div;", "return o;"),
    ("cookie interval closed", "pos < start[i] + (sigma - w[Blist[i]])", "pos <= start[i] + (sigma - w[Blist[i]])"),
    ("phi operands transposed", "if (pdn * cut < pn * cut_best) stall = 0;", "if (pn * cut < pdn * cut_best) stall = 0;"),
    ("balanced best never taken", "bal_best = 1; cut_best = cut; maxw_best = maxw; stall = 0;",
     "bal_best = 1; cut_best = cut; maxw_best = maxw;"),
    ("contraction keeps self loops", "if (cu == c) continue;", ""),
    ("rebalance from B side", "if (!inB[p] || conn[p] <= 0) continue;", "if (conn[p] <= 0) continue;"),
    ("ablation keeps locks", "locked[v] = (prm->flags & OG_F_NO_LOCKS) ? 0 : move[v];", "locked[v] = move[v];"),
    ("ablation still filters by F2", "if (prm->flags & OG_F_NO_AFTERBURNER) { move[v] = 1; nM++; continue; }", ""),
    ("two-hop leaves keyed by self", "kv[m].key = (uint64_t)(uint32_t)g->adjncy[g->xadj[v]];",
     "kv[m].key = (uint64_t)(uint32_t)v;"),
    ("two-hop pairs overlap", "for (int32_t a = i; a + 1 < j; a += 2) {", "for (int32_t a = i; a + 1 < j; a += 1) {"),
    ("two-hop never triggers", "if (4 * (int64_t)og_unmatched(match, n) <= (int64_t)n) break;", "break;"),
    ("start order ignores distance", "if (a->dist != b->dist) return a->dist < b->dist ? -1 : 1;\n", ""),
    ("start grows from largest id", "for (int32_t r = 0; r < n; r++) {\n        if (dist[r] >= 0) continue;",
     "for (int32_t r = n - 1; r >= 0; r--) {\n        if (dist[r] >= 0) continue;"),
    ("matching proposes the lightest edge", "if (bu < 0 || wt > bw ||", "if (bu < 0 || wt < bw ||"),
    ("matching ignores the round cap", "for (int32_t round = 0; round < 16; round++) {",
     "for (int32_t round = 0; round < 64; round++) {"),
    ("matching ignores the 1% rule", "if (newly == 0 || newly * 100 < (int64_t)n) break;", "if (newly == 0) break;"),
    ("coarse ids numbered by the larger member", "if (match[v] < 0 || v < match[v]) map[v] = nc++;",
     "if (match[v] < 0 || v > match[v]) map[v] = nc++;"),
    ("contraction overwrites edge weights", "acc[cu] += g->adjwgt[e];", "acc[cu] = g->adjwgt[e];"),
    ("projection ignores the map", "Pf[v] = P[maps[i][v]];", "Pf[v] = P[v % G[i + 1].n];"),
    ("coarsening target 4k", "G[nl - 1].n > 8 * (int64_t)k", "G[nl - 1].n > 4 * (int64_t)k"),
    ("coarsening drops the 90% rule", "if (nc == f->n || 10 * (int64_t)nc > 9 * (int64_t)f->n) { free(map); break; }",
     "if (nc == f->n) { free(map); break; }"),
    ("coarsening stops at 80%", "if (nc == f->n || 10 * (int64_t)nc > 9 * (int64_t)f->n) { free(map); break; }",
     "if (nc == f->n || 10 * (int64_t)nc > 8 * (int64_t)f->n) { free(map); break; }"),
    ("random start with the wrong stream", "og_mix64(prm->seed ^ 1ULL)", "og_mix64(prm->seed ^ 2ULL)"),
    ("start chunks by count", "        b += g->vwgt ? g->vwgt[v] : 1;\n    }\n    free(dist);",
     "        b += 1;\n    }\n    free(dist);"),
]

PIN_TESTS = [
    pins.test_golden_path4_refine,
    lambda O: pins.test_golden_rebalance(O, "path4_k2_jetrw.json", 2),
    lambda O: pins.test_golden_rebalance(O, "path6_k3_jetrs.json", 3),
    pins.test_slot_matches_bit_length,
    pins.test_gain_destination_against_sparse_product,
    pins.test_afterburner_equals_gain_under_expected_partition,
    pins.test_afterburner_independent_set_reduces_to_plain_gain,
    pins.test_c_filter_floor_boundaries,
    pins.test_rebalance_rules,
    pins.test_theorem1_bucket_prefix_loss_bound,
    pins.test_jetrw_balances_within_k_iterations_unit_weights,
    pins.test_jetrs_balances_in_one_iteration_unit_weights,
    pins.test_loop_invariants_and_brute_force,
    pins.test_stall_counter_follows_algorithm3,
    pins.test_exhaustive_optimum_bounds_result,
    pins.test_hem_is_a_matching_and_contraction_preserves_cut,
    pins.test_hem_path_closed_forms,
    pins.test_hem_distinct_weights_is_greedy_matching,
    pins.test_multilevel_is_algorithm1_composition,
    pins.test_partition_multilevel_sanity,
    pins.test_ablation_baseline_step_is_textbook_sync_lp,
    lambda O: pins.test_ablation_loop_iterates_textbook_lp(O, False),
    lambda O: pins.test_ablation_loop_iterates_textbook_lp(O, True),
    pins.test_two_hop_star_leaves_closed_form,
    pins.test_two_hop_isolated_vertices_never_pair,
    pins.test_two_hop_pairs_are_within_two_hops,
    pins.test_two_hop_passes_stop_once_three_quarters_match,
    pins.test_bfs_start_closed_forms,
    pins.test_bfs_start_against_library_bfs,
]


def _caught(libpath):
    with O.use_library(libpath):
        for t in PIN_TESTS:
            try:
                t(O)
            except (AssertionError, ValueError):
                return True
    return False


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site missing: {name}"
    mutated = src.replace(old, new, 1)
    cfile = tmp_path / "mut.c"
    cfile.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-std=gnu11", "-shared", "-fPIC", "-o", str(so), str(cfile)])
    assert _caught(str(so)), f"no pin caught the planted mistake: {name}"
