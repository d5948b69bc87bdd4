"""The oracle's pins must catch plausible mistakes: each case below plants
one mistake in a private copy of the oracle's C source (a dropped complement,
a skipped removal, an off-by-one row, a wrong branch set, a lost re-queue,
...), builds it into a temporary library and checks that the pin suite fails
against it.  Nothing here touches the GPU."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ct_oracle.c")

MUTANTS = [
    ("drop complement of incremental mask", "mask[w] = ~mask[w];", "mask[w] = mask[w];"),
    ("filter never removes", "if (!supported) dom[", "if (0) dom["),
    ("support row off by one", "(int64_t)(T->row_start[i] + a) * T->W",
     "(int64_t)(T->row_start[i] + a + (a > 0)) * T->W"),
    ("s_sup threshold", "if (size[i] > 1) {", "if (size[i] > 2) {"),
    ("delta reversed", "int take = incremental ? (was && !is) : is;",
     "int take = incremental ? (is && !was) : is;"),
    ("update stops after first variable", "if (T->kind == CTO_KIND_POSITIVE && !any_word(T->ct, W)) break;",
     "break;"),
    ("fixpoint never re-queues", "if (c2 == c || inq[c2]) continue;", "continue;"),
    ("OR instead of AND into currTable", "T->ct[w] &= mask[w];", "T->ct[w] |= mask[w];"),
    ("no stray-bit check", "int used = d - 64 * (T->dom_words[i] - 1);", "int used = 64;"),
    ("no subset check", "if (dom_in[k] & ~T->last_dom[k]) return CTO_E_NOT_SUBSET;", ";"),
    ("pop restores nothing", "memcpy(T->ct, T->snap_ct + (int64_t)T->depth * Wa, sizeof(uint64_t) * Wa);", ";"),
    # fast mode (sparse word list, residues, word trail)
    ("fast: emptied word stays listed", "                T->limit--;\n", "\n"),
    ("fast: removal swap dropped", "T->idx[k] = T->idx[T->limit - 1];", ";"),
    ("fast: no trail", "if (T->depth == 0 || T->stamp[w] == T->serial) return CTO_OK;", "return CTO_OK;"),
    ("fast: residue trusted without currTable", "if (T->ct[T->res[row]] & r[T->res[row]]) continue;",
     "if (r[T->res[row]]) continue;"),
    ("fast: mask ignores the last listed word",
     "for (int64_t k = 0; k < T->limit; k++) T->fmask[T->idx[k]] |= r[T->idx[k]];",
     "for (int64_t k = 0; k + 1 < T->limit; k++) T->fmask[T->idx[k]] |= r[T->idx[k]];"),
    ("fast: pop keeps the limit", "T->limit = T->lv_limit[T->depth];", ";"),
    # short and negative tables
    ("negative: product includes the filtered variable", "if (k == i) continue;", ";"),
    ("negative: removed values keep their tuples", "for (int64_t w = 0; w < T->W; w++) T->ct[w] &= ~r[w];", ";"),
    ("negative: unsupported iff count below the product", "if (cnt == prod) out[", "if (cnt < prod) out["),
    ("short: incremental branch ORs star rows",
     "const uint64_t *r = incremental ? strict_row_ptr(T, i, a) : row_ptr(T, i, a);",
     "const uint64_t *r = row_ptr(T, i, a);"),
    ("short: emptied domain on the incremental branch", "if (size == 0) return 0;", ";"),
    ("short: star cell supports no value", "for (int a = 0; a < dsz[i]; a++) row_ptr(T, i, a)[j / 64] |= 1ull << (j % 64);",
     ";"),
    # work counters
    ("rows selected counts the domain on both branches", "T->st[CTO_ST_ROWS_SEL] += incremental ? delta : size[i];",
     "T->st[CTO_ST_ROWS_SEL] += size[i];"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_kill_mutant(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site missing: {old}"
    mut = src.replace(old, new, 1)
    csrc = tmp_path / "mut.c"
    csrc.write_text(mut)
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-o", str(lib), str(csrc)],
                   check=True, capture_output=True)
    env = dict(os.environ, CT_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py"),
                        os.path.join(ROOT, "tests", "test_oracle_fast.py"),
                        os.path.join(ROOT, "tests", "test_oracle_kinds.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant survived the pins: {name}\n{r.stdout[-2000:]}"
