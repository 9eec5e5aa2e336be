"""The oracle's pins must catch plausible mistakes in the oracle.

Each case copies oracle/oracle.c, plants one mistake (a textual edit, on the
CPU), compiles the copy to a temporary library and runs the pin functions of
test_oracle.py against it: at least one pin must fail.
"""
import os

import numpy as np
import pytest

import oracle
from tests import test_oracle as T

MUTANTS = {
    "depth_plus_two": ("depth[v] = depth[u] + 1;", "depth[v] = depth[u] + 2;"),
    "lifo_queue": ("int32_t u = queue[head++];", "int32_t u = queue[--tail];"),
    "parent_is_self": ("        parent[v] = u;\n", "        parent[v] = (int32_t)v;\n"),
    "no_reverse_edge": ("    offsets[v + 1] += 1;\n", "\n"),
    "no_dedup": ("      if (i > start && adj[i] == adj[i - 1]) continue;\n", "\n"),
    "keeps_self_loops": ("    if (u == v) continue;\n    offsets[u + 1] += 1;",
                         "    offsets[u + 1] += 1;"),
    "validator_weak_level": ("if (depth_ref[p] != depth_ref[v] - 1) {",
                             "if (depth_ref[p] > depth_ref[v]) {"),
    "validator_no_edge_check": ("return lo < offsets[a + 1] && adj[lo] == b;", "return 1;"),
    "unionfind_no_union": ("        label[rb] = ra;", "        label[rb] = rb;"),
}

# Mistakes in the directed builder (several edits each), caught by the
# directed pins.
D_COUNT = "    if (u != v) offsets[u + 1] += 1;\n"
D_FILL = "    if (u != v) adj[fill[u]++] = v;\n"
DIRECTED_MUTANTS = {
    "directed_reversed": [(D_COUNT, "    if (u != v) offsets[v + 1] += 1;\n"),
                          (D_FILL, "    if (u != v) adj[fill[v]++] = u;\n")],
    "directed_symmetrised": [(D_COUNT, "    if (u != v) { offsets[u + 1] += 1; offsets[v + 1] += 1; }\n"),
                             (D_FILL, "    if (u != v) { adj[fill[u]++] = v; adj[fill[v]++] = u; }\n")],
    "directed_keeps_self_loops": [(D_COUNT, "    offsets[u + 1] += 1;\n"),
                                  (D_FILL, "    adj[fill[u]++] = v;\n")],
}


def pins_pass(L):
    from paper_1508_03619_amd import inputs
    if not T.exhaustive_depths_ok(L, 4):
        return False
    if not all(T.random_graph_ok(L, seed) for seed in range(12)):
        return False
    if not T.closed_forms_ok(L) or not T.golden_ok(L):
        return False
    el = inputs.rmat(10, 8, seed=3)
    if not T.invariants_ok(L, el, inputs.pick_sources(el, 3, seed=4)):
        return False
    return T.validator_ok(L)


def test_unmutated_oracle_passes_the_pins(oracle_lib):
    assert pins_pass(oracle_lib)


def _compile_mutant(tmp_path, edits):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    for old, new in edits:
        assert src.count(old) >= 1, f"mutation anchor missing: {old!r}"
        src = src.replace(old, new, 1)
    csrc = tmp_path / "oracle_mut.c"
    csrc.write_text(src)
    so = str(tmp_path / "liboracle_mut.so")
    import subprocess
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-o", so, str(csrc)], check=True)
    return oracle._bind(so)


@pytest.mark.parametrize("name", sorted(DIRECTED_MUTANTS))
def test_directed_mutant_is_caught(tmp_path, name):
    from tests import test_oracle_directed as TD
    L = _compile_mutant(tmp_path, DIRECTED_MUTANTS[name])
    try:
        caught = not TD.directed_pins_ok(L)
    except Exception:
        caught = True
    assert caught, f"mutant {name} passed every directed pin"


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(os.path.join(os.path.dirname(oracle.__file__), "oracle.c")).read()
    assert src.count(old) >= 1, f"mutation anchor missing for {name}"
    mutated = src.replace(old, new, 1)
    csrc = tmp_path / "oracle_mut.c"
    csrc.write_text(mutated)
    so = str(tmp_path / "liboracle_mut.so")
    import subprocess
    subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-std=c11", "-o", so, str(csrc)], check=True)
    L = oracle._bind(so)
    try:
        caught = not pins_pass(L)
    except Exception:
        caught = True  # a crash-free exception (e.g. bad input detected) also counts
    assert caught, f"mutant {name} passed every pin"


# Mistakes in the betweenness accumulation, caught by the betweenness pins.
BC_MUTANTS = {
    "bc_no_plus_one": [("* (1.0 + delta[v]);", "* (delta[v]);")],
    "bc_ratio_inverted": [("sigma[w] / sigma[v] *", "sigma[v] / sigma[w] *")],
    "bc_counts_predecessors": [("if (depth[v] == depth[u] + 1) sigma[v] += sigma[u];",
                                "if (depth[v] == depth[u] + 1) sigma[v] += 1.0;")],
    "bc_same_level_successor": [("        if (depth[v] == depth[w] + 1)\n          delta[w]",
                                 "        if (depth[v] >= depth[w])\n          delta[w]")],
    "bc_source_scored": [("      if (w != s) score[w] += delta[w];", "      score[w] += delta[w];")],
    "bc_normalise_by_sum": [("      if (score[v] > top) top = score[v];", "      top += score[v];")],
    "bc_sources_not_reset": [("      sigma[v] = 0.0;\n      delta[v] = 0.0;", "      sigma[v] = 0.0;")],
}


@pytest.mark.parametrize("name", sorted(BC_MUTANTS))
def test_bc_mutant_is_caught(tmp_path, name):
    from tests import test_oracle_bc as TB
    L = _compile_mutant(tmp_path, BC_MUTANTS[name])
    assert not TB.bc_pins_ok(L), f"mutant {name} passed every betweenness pin"


# Mistakes in the weighted builder and Dijkstra, caught by the shortest-path pins.
SSSP_MUTANTS = {
    "sssp_keeps_heaviest_repeat": [("  return (x->w > y->w) - (x->w < y->w);",
                                    "  return (x->w < y->w) - (x->w > y->w);")],
    "sssp_ignores_weights": [("      const int64_t nd = it.d + wadj[i];", "      const int64_t nd = it.d + 1;")],
    "sssp_max_heap": [("    if (h[p].d <= d) break;", "    if (h[p].d >= d) break;"),
                      ("    if (c + 1 < *size && h[c + 1].d < h[c].d) ++c;\n    if (h[c].d >= last.d) break;",
                       "    if (c + 1 < *size && h[c + 1].d > h[c].d) ++c;\n    if (h[c].d <= last.d) break;")],
    "sssp_no_reverse_edge": [("    if (!directed) {\n      tmp[fill[v]].v = u;", "    if (0) {\n      tmp[fill[v]].v = u;")],
    "sssp_first_visit_final": [("      if (!done[v] && (dist[v] < 0 || nd < dist[v])) {",
                                "      if (!done[v] && dist[v] < 0) {")],
}


@pytest.mark.parametrize("name", sorted(SSSP_MUTANTS))
def test_sssp_mutant_is_caught(tmp_path, name):
    from tests import test_oracle_sssp as TS
    L = _compile_mutant(tmp_path, SSSP_MUTANTS[name])
    assert not TS.sssp_pins_ok(L), f"mutant {name} passed every shortest-path pin"


# Mistakes in union-find and the component verifier, caught by the CC pins.
CC_MUTANTS = {
    "cc_larger_root_wins": [("      if (ra < rb)\n        label[rb] = ra;\n      else\n        label[ra] = rb;",
                             "      if (ra > rb)\n        label[rb] = ra;\n      else\n        label[ra] = rb;")],
    "cc_skips_last_edge": [("  for (int64_t e = 0; e < m; ++e) {\n    int32_t a = src[e], b = dst[e];\n    if (a < 0",
                            "  for (int64_t e = 0; e + 1 < m; ++e) {\n    int32_t a = src[e], b = dst[e];\n    if (a < 0")],
    "cc_check_ignores_reuse": [("    if (used[h] == (int64_t)L) {\n      rc = 2;", "    if (0) {\n      rc = 2;")],
}


@pytest.mark.parametrize("name", sorted(CC_MUTANTS))
def test_cc_mutant_is_caught(tmp_path, name):
    from tests import test_oracle_cc as TC
    L = _compile_mutant(tmp_path, CC_MUTANTS[name])
    assert not TC.cc_pins_ok(L), f"mutant {name} passed every component pin"
