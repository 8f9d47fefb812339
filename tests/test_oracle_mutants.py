"""Planted mistakes in copies of the oracle must each fail a pin (CPU only).

Each mutant is a textual edit of oracle/oracle.cpp compiled into a temporary
library; the pins (hand fixtures, closed forms, brute force, the O(n^2) stream
definition, the digest's known answer and word coverage) are re-run against it and at least one must fail.  The original
snippet must still be present, so the list follows the oracle as it changes.
"""
import os
import subprocess

import numpy as np
import pytest

import gen
import oracle
from oracle.brute import brute
from oracle.closed_form import cyclic_capped, cyclic_summary

from conftest import ROOT, load_golden, model_from_fixture, result_fields
from test_oracle_pins import FNV_TO_SPLITMIX_SEED0, SPLITMIX64_SEED0_FIRST, _digest_sees_every_word

MUTANTS = [
    ("guard reads a local instead of the shared var",
     "s[m.P + t[1]] != t[2]", "s[t[1]] != t[2]"),
    ("guard polarity inverted", "s[m.P + t[1]] != t[2]", "s[m.P + t[1]] == t[2]"),
    ("effect dropped", "out[o + m.P + t[3]] = t[4];", "(void)0;"),
    ("effect written to a local", "out[o + m.P + t[3]] = t[4];", "out[o + t[3]] = t[4];"),
    ("local step dropped", "out[o + p] = t[0];", "(void)0;"),
    ("edges count states, not successors", "lvl_edges += n;", "lvl_edges += (n != 0);"),
    ("deadlock test inverted", "lvl_dead += (n == 0);", "lvl_dead += (n != 0);"),
    ("cap off by one", "cap && a.rows() > cap", "cap && a.rows() >= cap"),
    ("edges of the discarded level kept", "sum->capped = 1;", "sum->capped = 1; sum->edges += lvl_edges;"),
    ("queue-if-seen polarity", "if (!V.insert(cand).second)", "if (V.insert(cand).second)"),
    ("transition table index transposed",
     "((static_cast<uint64_t>(p) * L + l) * K + k) * 5",
     "((static_cast<uint64_t>(l) * P + p) * K + k) * 5"),
    ("level count off by one", "level_counts[sum->n_levels++] = fresh;",
     "level_counts[sum->n_levels++] = fresh + (fresh > 3);"),
    ("stream seen polarity", "seen[k] = 1;", "seen[k] = 0;"),
    ("stream id of repeat", "id[k] = it->second;", "id[k] = static_cast<uint32_t>(distinct - 1);"),
    ("digest skips the last word", "for (uint32_t i = 0; i < W; ++i) {\n        h ^= r[i];",
     "for (uint32_t i = 0; i < W - 1; ++i) {\n        h ^= r[i];"),
    ("digest reads half the row", "for (uint32_t i = 0; i < W; ++i) {\n        h ^= r[i];",
     "for (uint32_t i = 0; i < W / 2; ++i) {\n        h ^= r[i];"),
    ("digest reads one word over and over", "h ^= r[i];", "h ^= r[0];"),
    ("digest finaliser step dropped", "h ^= h >> 27;", "(void)0;"),
    ("set digest keeps only the last row", "s += d;", "s = d;"),
]


def _pins_pass(lib) -> bool:
    saved = oracle._lib
    oracle._lib = lib
    try:
        for fx in load_golden("reach_fixtures.json")["fixtures"]:
            m = model_from_fixture(fx)
            for case in fx["cases"]:
                want = {k: case[k] for k in ("total", "level_counts", "edges", "deadlocks", "capped")}
                want["n_levels"] = len(case["level_counts"])
                if result_fields(oracle.reach(m, cap=case["cap"])) != want:
                    return False
        for N, L in [(2, 3), (3, 4), (4, 8)]:
            m = gen.cyclic_model(N, L)
            if result_fields(oracle.reach(m, cap=0)) != cyclic_summary(N, L):
                return False
            if result_fields(oracle.reach(m, cap=L ** N // 3)) != cyclic_capped(N, L, L ** N // 3):
                return False
        rng = np.random.default_rng(3)
        for i in range(40):
            m = gen.guarded_model(500 + i, int(rng.integers(1, 4)), int(rng.integers(2, 5)),
                                  int(rng.integers(1, 3)), int(rng.integers(2, 4)), int(rng.integers(1, 4)))
            b = brute(m, cap=0)
            if result_fields(oracle.reach(m, cap=0)) != b:
                return False
        if oracle.digest(np.array([FNV_TO_SPLITMIX_SEED0], dtype=np.uint32)) != \
                (1, SPLITMIX64_SEED0_FIRST, SPLITMIX64_SEED0_FIRST):
            return False
        for W in (1, 2, 17, 32):
            if not _digest_sees_every_word(W):
                return False
        for fx in load_golden("stream_fixtures.json")["fixtures"]:
            seen, ids, d = oracle.stream(np.array(fx["rows"], dtype=np.uint32))
            if seen.tolist() != fx["seen"] or ids.tolist() != fx["id"] or d != fx["distinct"]:
                return False
        return True
    except Exception:
        return False
    finally:
        oracle._lib = saved


def test_unmutated_oracle_passes_pins():
    assert _pins_pass(oracle.lib())


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(tmp_path, name, orig, mut):
    src = open(os.path.join(ROOT, "oracle", "oracle.cpp")).read()
    assert orig in src, f"mutant anchor missing: {orig}"
    path = tmp_path / "mut.cpp"
    path.write_text(src.replace(orig, mut, 1))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", str(path), "-o", str(so)])
    assert not _pins_pass(oracle.load(str(so))), f"pins did not catch: {name}"
