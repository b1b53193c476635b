"""The pins must be sharp enough to catch plausible mistakes in the oracle.

Each case below plants one mistake in a private copy of ``oracle_fw.c``
(a dropped term, a wrong index, a transposed operand, a lost tie-break...),
compiles it with gcc into a temporary library and runs a battery of pins
against it: at least one pin must fail.  The real oracle must pass the same
battery.  Everything runs on the CPU."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import pins

INF32 = pins.INF32
SRC = open(oracle.SRC_PATH).read()

MUTANTS = {
    "non_strict_compare": ("if (s < d) {\n                    di[j] = (int32_t)s;",
                           "if (s <= d) {\n                    di[j] = (int32_t)s;"),
    "transposed_column_read": ("const int64_t a = D[i * n + k];", "const int64_t a = D[k * n + i];"),
    "no_inf_absorption": ("if (a == ORC_INF || b == ORC_INF) return ORC_INF;", ""),
    "intermediate_node_pred": ("if (pi) pi[j] = prow[j];\n                } else if (pi && s == d && s != ORC_INF",
                               "if (pi) pi[j] = (int32_t)k;\n                } else if (pi && s == d && s != ORC_INF"),
    "dropped_last_iteration": ("int st = oracle_fw_i32_steps(D, P, n, 0, n, threads);",
                               "int st = oracle_fw_i32_steps(D, P, n, 0, n - 1, threads);"),
    "no_tie_break": ("} else if (pi && s == d && s != ORC_INF && prow[j] < pi[j]) {",
                     "} else if (0) {"),
    "tie_break_wrong_way": ("} else if (pi && s == d && s != ORC_INF && prow[j] < pi[j]) {",
                            "} else if (pi && s == d && s != ORC_INF && prow[j] > pi[j]) {"),
    "pred_init_wrong_owner": ("? (int32_t)i : ORC_NONE;\n}\n\nvoid oracle_pred_init_f64",
                              "? (int32_t)j : ORC_NONE;\n}\n\nvoid oracle_pred_init_f64"),
    "pred_from_first_half": ("if (pi) pi[j] = prow[j];\n                } else if (pi && s == d && s != ORC_INF",
                             "if (pi) pi[j] = pi[k];\n                } else if (pi && s == d && s != ORC_INF"),
    "diag_pred_not_cleared": ("if (i == j || D[i * n + j] == ORC_INF || P[i * n + j] == ORC_NONE)\n                    P[i * n + j] = -1;\n    return status;\n}\n\nint oracle_finalize_f64",
                              "if (D[i * n + j] == ORC_INF)\n                    P[i * n + j] = -1;\n    return status;\n}\n\nint oracle_finalize_f64"),
    "negative_cycle_missed": ("if (D[i * n + i] < 0) status = ORC_NEGATIVE_CYCLE;\n    if (P)\n        for (int64_t i = 0; i < n; ++i)\n            for (int64_t j = 0; j < n; ++j)\n                if (i == j || D[i * n + j] == ORC_INF",
                              "if (D[i * n + i] < -1000000) status = ORC_NEGATIVE_CYCLE;\n    if (P)\n        for (int64_t i = 0; i < n; ++i)\n            for (int64_t j = 0; j < n; ++j)\n                if (i == j || D[i * n + j] == ORC_INF"),
    "row_wrong_sign": ("const int64_t s = sat_add(dist[u], wu[v]);", "const int64_t s = sat_add(dist[u], -wu[v]);"),
    "row_pred_last_match": ("if (j == v || prow[j] != ORC_NONE || wv[j] == ORC_INF || dist[j] == ORC_INF)",
                            "if (j == v || wv[j] == ORC_INF || dist[j] == ORC_INF)"),
}


def battery(orc) -> list:
    """Return the names of the pins that fail for this oracle library."""
    failed = []
    rng = np.random.default_rng(2024)
    # brute force, ties (small weights) and negative weights (potential graphs)
    ok = True
    for t in range(24):
        n = 3 + t % 4
        W = pins.random_graph(rng, n, 0.6, 1, 3 if t % 2 else 50, potential=(t % 3 == 0))
        D, P, st = orc.fw(W, pred=True)
        bd, bp = pins.brute_force(W)
        if st != 0 or [[None if x == INF32 else int(x) for x in r] for r in D] != bd or P.tolist() != bp:
            ok = False
            break
    if not ok:
        failed.append("brute_force")
    # Dijkstra + canonical predecessor on a medium graph
    W = pins.random_graph(rng, 60, 0.1, 1, 20)
    D, P, _ = orc.fw(W, pred=True)
    for i in (0, 17, 59):
        dr = pins.dijkstra_row(W, i)
        if [None if x == INF32 else int(x) for x in D[i]] != dr or \
                P[i].tolist() != pins.canonical_pred_row(W, dr, i):
            failed.append("dijkstra")
            break
    # negative cycle detection
    Wn = np.full((3, 3), INF32, dtype=np.int32)
    np.fill_diagonal(Wn, 0)
    Wn[0, 1], Wn[1, 2], Wn[2, 0] = 1, 1, -3
    if orc.fw(Wn)[2] != oracle.NEGATIVE_CYCLE:
        failed.append("negative_cycle")
    # row oracle against Dijkstra / Bellman-Ford
    Wp = pins.random_graph(rng, 50, 0.2, 1, 9, potential=True)
    for src in (0, 25):
        dr, pr, st = orc.row(Wp, src, pred=True)
        bf, _ = pins.bellman_ford_row(Wp, src)
        if [None if x == INF32 else int(x) for x in dr] != bf or \
                pr.tolist() != pins.canonical_pred_row(Wp, bf, src):
            failed.append("row")
            break
    return failed


def test_real_oracle_passes_battery(orc):
    assert battery(orc) == []


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    return tmp_path_factory.mktemp("mutants")


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, workdir):
    old, new = MUTANTS[name]
    assert SRC.count(old) == 1, f"mutation anchor for {name} not unique/present"
    src = os.path.join(workdir, f"{name}.c")
    so = os.path.join(workdir, f"lib{name}.so")
    with open(src, "w") as f:
        f.write(SRC.replace(old, new))
    subprocess.check_call(["gcc", "-O1", "-fPIC", "-shared", "-fopenmp", "-o", so, src, "-lm"])
    orc = oracle.Oracle(oracle.load(so))
    assert battery(orc) != [], f"mutant {name} survived every pin"
