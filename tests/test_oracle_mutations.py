"""Planted mistakes in a copy of the oracle must be caught by the pins.

Each case copies ``oracle/wt_oracle.c`` to a temporary directory, applies one
plausible mistake (a swapped order, a dropped condition, an off-by-one, a
wrong bit order), compiles it with gcc and runs every pin against it.  At
least one pin must fail; otherwise the pins would not protect the oracle from
that kind of error.  Runs on the CPU only.
"""
import json
import os
import shutil
import subprocess
import sys

import pytest

import oracle
from tests import pins

MUTATIONS = {
    # WM partition puts ones first
    "wm_ones_first": ("uint64_t z = 0, o = nz;", "uint64_t z = n - nz, o = 0;"),
    # WT partition ignores the node boundaries (becomes a WM-like global split)
    "wt_global_split": ("while (b < n && prefix_of(L, l, seq[b]) == p) {", "while (b < n) {"),
    # bits read LSB-first instead of MSB-first
    "lsb_first": ("return (uint32_t)(((uint64_t)a >> (L - 1 - k)) & 1u);",
                  "return (uint32_t)(((uint64_t)a >> k) & 1u);"),
    # prefix one bit too short
    "prefix_short": ("return (uint64_t)a >> (L - k);", "return (uint64_t)a >> (L - k + 1);"),
    # Z counts ones
    "z_counts_ones": ("if (bit_of(L, l, seq[i])) set_bit(lv, i);\n            else nz++;",
                      "if (bit_of(L, l, seq[i])) { set_bit(lv, i); nz++; }"),
    # WM interval order without the bit reversal
    "spos_no_reverse": ("uint64_t p = (kind == ORC_WT) ? i : orc_reverse_bits(i, level);",
                        "uint64_t p = i;"),
    # inclusive rank
    "rank_inclusive": ("for (uint64_t p = 0; p < i; p++)\n        if (get_bit(words, p) == b) c++;",
                       "for (uint64_t p = 0; p <= i; p++)\n        if (get_bit(words, p) == b) c++;"),
    # select returns the (k+1)-th
    "select_off_by_one": ("if (c == k) return p;", "if (c == k + 1) return p;"),
    # directory block boundary off by one bit
    "rank_dir_short_block": ("p < 512 * (j + 1) && p < n;", "p < 512 * (j + 1) - 1 && p < n;"),
    # select samples every 4096 zeros taken from the ones
    "sel0_from_ones": ("if (c0 % ORC_SEL_SPACING == 0) sel0[c0 / ORC_SEL_SPACING] = (uint32_t)(p / 512);",
                       "if (c1 % ORC_SEL_SPACING == 0) sel0[c1 / ORC_SEL_SPACING] = (uint32_t)(p / 512);"),
    # histogram counted on the prefix one level deeper
    "hist_wrong_level": ("hist[prefix_of(L, level, sym_at(text, sym_bytes, i))]++;",
                         "hist[prefix_of(L, level, sym_at(text, sym_bytes, i)) >> 1]++;"),
    # symbol range check missing
    "no_range_check": ("if (L < 32 && (a >> L) != 0) return ORC_ERANGE;", "(void)a;"),
    # WT rank walk maps the zero child with the wrong base
    "walk_wt_rank_base": ("p = s + orc_rank_bv(lv, p, 0) - r0s;", "p = orc_rank_bv(lv, p, 0) - r0s;"),
    # position map takes the WM start from the WT order
    "map_wm_start_from_wt": ("out[q] = swm[lo] + (i - swt[lo]);", "out[q] = swt[lo] + (i - swt[lo]);"),
    # position map searches with the WM starts
    "map_search_wm_order": ("if (swt[mid] <= i) lo = mid;", "if (swm[mid] <= i) lo = mid;"),
    # pointer tree: runs of floor instead of ceil words (overlapping nodes)
    "ptree_runs_floor": ("w += (nodes[2 * e + 1] + 63) / 64;", "w += nodes[2 * e + 1] / 64;"),
    # pointer tree: nodes of a level in bit-reversed (WM) order
    "ptree_reversed_nodes": ("uint64_t e = ((uint64_t)1 << l) - 1 + prefix_of(L, l, a);",
                             "uint64_t e = ((uint64_t)1 << l) - 1 + orc_reverse_bits(prefix_of(L, l, a), l);"),
    # pointer tree: bits of a node in reverse text order
    "ptree_reverse_text": ("uint64_t q = fill[e]++;", "uint64_t q = nodes[2 * e + 1] - 1 - fill[e]++;"),
    # one-scan rank counts T[0, i] instead of T[0, i)
    "rank_scan_inclusive": ("while (i < p) count[sym_at(text, sym_bytes, i++)]++;",
                            "while (i <= p && i < n) count[sym_at(text, sym_bytes, i++)]++;"),
    # one-scan rank answers in the sorted order instead of the caller's
    "rank_scan_sorted_order": ("out[q] = (syms[q] < sigma_end) ? count[syms[q]] : 0;",
                               "out[r] = (syms[r] < sigma_end) ? count[syms[r]] : 0;"),
    # WM select walk forgets the Z offset
    "walk_wm_select_z": ("p = b ? orc_select_bv(lv, n, p - zeros[l] + 1, 1)", "p = b ? orc_select_bv(lv, n, p + 1, 1)"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    src_dir = os.path.dirname(oracle.__file__)
    src = open(os.path.join(src_dir, "wt_oracle.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    shutil.copy(os.path.join(src_dir, "wt_oracle.h"), tmp_path / "wt_oracle.h")
    (tmp_path / "wt_oracle.c").write_text(src.replace(old, new))
    lib = oracle.compile_library(str(tmp_path / "wt_oracle.c"), str(tmp_path / "libmut.so"))
    # the mutant may corrupt memory, so its pins run in a child process
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import json, sys\n"
        f"sys.path.insert(0, {root!r})\n"
        "import oracle\n"
        "from tests import pins\n"
        f"m = oracle.Oracle({lib!r})\n"
        "failed = []\n"
        "for check in pins.ALL_CHECKS:\n"
        "    try:\n"
        "        if check is pins.check_levels_brute:\n"
        "            check(m, exhaustive=False)\n"
        "        else:\n"
        "            check(m)\n"
        "    except Exception:\n"
        "        failed.append(check.__name__)\n"
        "        print(json.dumps(failed), flush=True)\n"
        "print(json.dumps(failed), flush=True)\n"
    )
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    lines = [ln for ln in r.stdout.splitlines() if ln.startswith("[")]
    failed = json.loads(lines[-1]) if lines else []
    # a pin that fails, or a mutant that crashes before any pin finishes, is caught
    assert failed or r.returncode != 0, f"no pin caught the planted mistake {name}"


# planted mistakes in the all-cores builder (wt_oracle_par.c)
PAR_MUTATIONS = {
    # threads' destinations handed out in reverse thread order (unstable)
    "par_threads_reversed": ("for (int t = 0; t < T; t++) {\n                uint64_t *c = cnt + ((uint64_t)t * nodes + k) * 2;",
                             "for (int t = T - 1; t >= 0; t--) {\n                uint64_t *c = cnt + ((uint64_t)t * nodes + k) * 2;"),
    # the ones of a node start right after the node's start (zeros overwritten)
    "par_ones_at_node_start": ("uint64_t zc = run, oc = run + z;", "uint64_t zc = run, oc = run;"),
    # the WT split ignores the nodes (a WM-like global split)
    "par_wt_no_nodes": ("const uint64_t node = (kind == ORC_WT && l > 0) ? (a >> (L - l)) : 0;\n                tmp",
                        "const uint64_t node = 0;\n                tmp"),
}


@pytest.mark.parametrize("name", sorted(PAR_MUTATIONS))
def test_planted_mistake_in_par_builder_is_caught(tmp_path, name):
    old, new = PAR_MUTATIONS[name]
    src_dir = os.path.dirname(oracle.__file__)
    src = open(os.path.join(src_dir, "wt_oracle_par.c")).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    shutil.copy(os.path.join(src_dir, "wt_oracle.h"), tmp_path / "wt_oracle.h")
    (tmp_path / "wt_oracle_par.c").write_text(src.replace(old, new))
    par = oracle.compile_par_library(str(tmp_path / "wt_oracle_par.c"), str(tmp_path / "libmutpar.so"))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys\n"
        f"sys.path.insert(0, {root!r})\n"
        "import oracle\n"
        "from tests import pins\n"
        f"m = oracle.Oracle(oracle._LIB, par_path={par!r})\n"
        "try:\n"
        "    pins.check_par_build(m)\n"
        "except Exception:\n"
        "    print('CAUGHT', flush=True)\n"
    )
    oracle.load()  # the single-threaded oracle, compiled if needed
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert "CAUGHT" in r.stdout or r.returncode != 0, f"no pin caught the planted mistake {name}"
