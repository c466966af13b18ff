"""Planted mistakes in the oracle, each caught by one of its pins.

Every case copies oracle/hsga_oracle.c, plants one plausible mistake by a
textual edit, builds the copy with gcc and calls the listed pins (test
functions of the other test_oracle_* files) with the planted copy in place
of the oracle: at least one of them must fail.  This is the evidence that
each part of the oracle is pinned to something other than itself -- a
mistake that no pin catches would be shared silently by a kernel written
from the same misreading.

Not listed, because no property of the paper can tell them apart: the
conventions of the random-number mapping (which Philox word plays which
role, which draw wins a tie, the order in which the four directions'
immigrants are written).  Any choice gives the same law; these are fixed by
the reading alone, and the GPU path is compared with it word for word.
"""
import importlib.util
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE_C = os.path.join(ROOT, "oracle", "hsga_oracle.c")
ORACLE_PY = os.path.join(ROOT, "oracle", "hsga_oracle.py")

# name -> (text in the oracle, planted replacement, [(pin module, pin, kwargs)])
MUTANTS = {
    "placement takes the highest evictable site": (
        "    for (uint32_t k = 0; k < m; k++) {\n        uint32_t tg = L[offset + k];",
        "    for (uint32_t kk = 0; kk < m; kk++) {\n        uint32_t k = m - 1 - kk;\n"
        "        uint32_t tg = L[offset + k];",
        [("test_oracle_site_vectors", "test_vectors_match_oracle", {})]),
    "steady spacing one bit too wide": (
        "uint64_t spacing = (uint64_t)1 << bitlen64(q);",
        "uint64_t spacing = (uint64_t)1 << (bitlen64(q) + 1);",
        [("test_oracle_site_rule", "test_steady_criteria", {"m": 8})]),
    "tilted keeps one item fewer per level": (
        "return c + r >= n_h;",
        "return c + r > n_h;",
        [("test_oracle_site_rule", "test_tilted_criteria", {"m": 8})]),
    "hybrid runs the tilted policy on both halves": (
        "*policy = ORC_STEADY; *u = T / 2; *offset = 0;",
        "*policy = ORC_TILTED; *u = T / 2; *offset = 0;",
        [("test_oracle_site_rule", "test_hybrid_is_half_steady_half_tilted", {"S": 32})]),
    "tournament compares traits unsigned": (
        "if ((int32_t)q->trait[b] > (int32_t)q->trait[p])",
        "if (q->trait[b] > q->trait[p])",
        [("test_oracle_ga", "test_selection_raises_mean_trait", {})]),
    "tournament keeps the lower trait": (
        "if ((int32_t)q->trait[b] > (int32_t)q->trait[p])",
        "if ((int32_t)q->trait[b] < (int32_t)q->trait[p])",
        [("test_oracle_ga", "test_selection_raises_mean_trait", {})]),
    "mutation range one value too wide": (
        "(int32_t)orc_mulhi(w[3], r->mut_span) + r->mut_lo",
        "(int32_t)orc_mulhi(w[3], r->mut_span + 1) + r->mut_lo",
        [("test_oracle_ga", "test_mutation_statistics", {})]),
    "differentia written one site off": (
        "        if (ingest) {\n            uint32_t per_word = 32 / r->bits;\n"
        "            uint32_t shift = ((uint32_t)site % per_word) * r->bits;",
        "        if (ingest) {\n            uint32_t per_word = 32 / r->bits;\n"
        "            uint32_t shift = ((uint32_t)(site ^ 1) % per_word) * r->bits;",
        [("test_oracle_ga", "test_pedigree_consistency", {"kind": 0})]),
    "immigrants never written into the island": (
        "    if (r->migrants && r->has_outbox) {\n"
        "        orc_philox(0, i, g, ORC_IMMIGRATE, r->seed, w);",
        "    if (0 && r->migrants && r->has_outbox) {\n"
        "        orc_philox(0, i, g, ORC_IMMIGRATE, r->seed, w);",
        [("test_oracle_ga", "test_immigrants_become_parents", {})]),
    "emigrants sent north or south only": (
        "    uint32_t a = i * N + e;\n    r->ob_dir[i] = w[1] >> 30;\n",
        "    uint32_t a = i * N + e;\n    r->ob_dir[i] = w[1] >> 31;\n",
        [("test_oracle_ga", "test_emigrant_directions_are_uniform", {})]),
    "MRCA upper bound at the last agreeing item": (
        "            *ub = gen;\n            *lb = have_last ? last + 1 : 0;",
        "            *ub = have_last ? last : 0;\n            *lb = have_last ? last + 1 : 0;",
        [("test_oracle_mrca", "test_bounds_against_true_pedigree",
          {"kind": 1, "S": 32, "tournament": 0})]),
    "MRCA lower bound without the +1": (
        "    *ub = Ta < Tb ? Ta : Tb;\n    *lb = have_last ? last + 1 : 0;",
        "    *ub = Ta < Tb ? Ta : Tb;\n    *lb = have_last ? last : 0;",
        [("test_oracle_mrca", "test_hand_built_fill_phase_annotations", {})]),
    "sample stratum one agent too wide": (
        "idx[k] = lo + orc_mulhi(w[0], hi - lo);",
        "idx[k] = lo + orc_mulhi(w[0], hi - lo + 1);",
        [("test_oracle_mrca", "test_stratified_sample", {"A": 7, "n": 3}),
         ("test_oracle_mrca", "test_stratified_sample", {"A": 2048, "n": 1024})]),
    "half-normal: wrong fourth cosine coefficient": (
        "1.0, -1.0 / 2.0, 1.0 / 24.0, -1.0 / 720.0, 1.0 / 40320.0,",
        "1.0, -1.0 / 2.0, 1.0 / 24.0, -1.0 / 721.0, 1.0 / 40320.0,",
        [("test_oracle_float", "test_half_normal_exact_to_1e14", {})]),
    "deleterious mutations raise fitness": (
        "child_trait = f32_bits((float)(f - (double)r->del_sigma *",
        "child_trait = f32_bits((float)(f + (double)r->del_sigma *",
        [("test_oracle_float", "test_purifying_only_never_gains", {})]),
    "asynchronous child counter taken from the tick": (
        "            r->n_counter[a] = T + 1;\n            for (uint32_t s = 0; s < SW; s++)\n"
        "                r->n_surf[(size_t)a * SW + s] = q->surf[p * SW + s];\n"
        "            if (T % r->interval == 0) {",
        "            r->n_counter[a] = k + 1;\n            for (uint32_t s = 0; s < SW; s++)\n"
        "                r->n_surf[(size_t)a * SW + s] = q->surf[p * SW + s];\n"
        "            if (T % r->interval == 0) {",
        [("test_oracle_async", "test_births_raise_the_parents_own_counter", {})]),
    "tree leaf edges left out of the branch length": (
        "            if (k == 1 && has_parent) {\n                c->sbl += c->T - parent_t;",
        "            if (k == 1 && has_parent) {\n                c->sbl += 0;",
        [("test_oracle_phylo", "test_hand_worked_tree", {})]),
    "tree pairs meet at the parent's time": (
        "c->pair_sum += seen * k * (uint64_t)(c->T - here);",
        "c->pair_sum += seen * k * (uint64_t)(c->T - (has_parent ? parent_t : here));",
        [("test_oracle_phylo", "test_hand_worked_tree", {})]),
}


def _load_module(name, path):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.fixture(scope="module")
def pin_modules():
    return {}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
@pytest.mark.parametrize("name", list(MUTANTS))
def test_planted_mistake_is_caught(tmp_path, name, pin_modules):
    old, new, pins = MUTANTS[name]
    with open(ORACLE_C) as f:
        src = f.read()
    assert src.count(old) == 1, f"the text to plant into is not unique in the oracle: {name}"
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-pthread", "-w", "-shared", "-fPIC",
                    "-o", str(lib), str(mutant_c), "-lm"], check=True)
    mut = _load_module(f"orc_mutant_{abs(hash(name))}", ORACLE_PY)
    mut.LIB = str(lib)
    mut.load()
    caught = []
    for mod_name, pin, kwargs in pins:
        if mod_name not in pin_modules:
            pin_modules[mod_name] = _load_module(f"pins_{mod_name}",
                                                 os.path.join(HERE, mod_name + ".py"))
        fn = getattr(pin_modules[mod_name], pin)
        try:
            fn(mut, **kwargs)
        except (AssertionError, ValueError, RuntimeError):
            caught.append(pin)
    assert caught, f"no pin caught the planted mistake: {name}"
