"""Plant plausible mistakes in copies of the C oracle (on the CPU) and check
that the pin suite catches every one of them."""
import os
import shutil
import subprocess

import pytest

import oracle
from tests.oracle_pins import ALL_PINS

SRC = os.path.join(os.path.dirname(oracle.__file__), "lb_oracle.c")

# (name, text in lb_oracle.c, replacement)
MUTANTS = [
    ("drop_last_term", "for (int64_t j = row_offsets[r]; j < row_offsets[r + 1]; ++j) {\n            double t = orc_load(values, vdt, j) * orc_load(x, xdt, col_idx[j]);",
     "for (int64_t j = row_offsets[r]; j < row_offsets[r + 1] - 1; ++j) {\n            double t = orc_load(values, vdt, j) * orc_load(x, xdt, col_idx[j]);"),
    ("row_for_col", "double t = orc_load(values, vdt, j) * orc_load(x, xdt, col_idx[j]);",
     "double t = orc_load(values, vdt, j) * orc_load(x, xdt, col_idx[j] ^ (j & 1 ? 0 : (col_idx[j] > 0)));"),
    ("sign_flip", "sum += abs_terms ? (t < 0 ? -t : t) : t;\n        }\n        y[r] = sum;",
     "sum += abs_terms ? (t < 0 ? -t : t) : (j == row_offsets[r] ? -t : t);\n        }\n        y[r] = sum;"),
    ("accumulate_y", "        y[r] = sum;", "        y[r] += sum;"),
    ("spmm_bad_index", "orc_load(X, xdt, (int64_t)col_idx[j] * ldx + c)", "orc_load(X, xdt, (int64_t)j % (k ? k : 1) * 0 + (int64_t)col_idx[j] * ldx)"),
    ("transpose_uses_row", "dx[col_idx[j]] += abs_terms", "dx[col_idx[j] == 0 ? 0 : col_idx[j] - (r & 1)] += abs_terms"),
    ("dvalues_wrong_row", "dvalues[j] = dy[r] * orc_load(x, xdt, col_idx[j]);", "dvalues[j] = dy[r > 0 ? r - 1 : 0] * orc_load(x, xdt, col_idx[j]);"),
    ("merge_tie_nnz_first", "if (i < m && row_offsets[i + 1] <= j)", "if (i < m && row_offsets[i + 1] < j)"),
    ("merge_off_by_one", "int64_t target = t * W < total ? t * W : total;", "int64_t target = t * W + 1 < total ? t * W + 1 : total;"),
    ("sssp_wrong_weight_index", "float offer = dist[u] + w[j];", "float offer = dist[u] + w[row_offsets[u]];"),
    ("sssp_dropped_weight", "float offer = dist[u] + w[j];", "float offer = dist[u] + (j & 1 ? w[j] : 0.0f);"),
    ("sssp_wrong_endpoint", "int32_t v = col_idx[j];\n            float offer", "int32_t v = (j % 3 == 0 && col_idx[j] > 0) ? col_idx[j] - 1 : col_idx[j];\n            float offer"),
    ("sssp_stop_early", "while (size > 0) {", "while (size > 1) {"),
    ("bfs_dropped_increment", "depth[v] = depth[u] + 1;", "depth[v] = depth[u] + (u != source);"),
    ("bfs_stack_not_queue", "int32_t u = queue[head++];", "int32_t u = queue[--tail];"),
    ("coo_wrong_row", "        y[row_idx[j]] += abs_terms ? (t < 0 ? -t : t) : t;\n    }\n    return 0;\n}\n\n/* CSC",
     "        y[row_idx[j] > 0 && (j & 1) ? row_idx[j] - 1 : row_idx[j]] += abs_terms ? (t < 0 ? -t : t) : t;\n    }\n    return 0;\n}\n\n/* CSC"),
    ("csc_wrong_x", "double xc = orc_load(x, xdt, c);", "double xc = orc_load(x, xdt, c > 0 && (c & 1) ? c - 1 : c);"),
    ("spgemm_wrong_b_entry", "double t = a * orc_load(b_val, bdt, f);", "double t = a * orc_load(b_val, bdt, f > b_ro[j] ? f - 1 : f);"),
    ("spgemm_skips_first_column", "                int32_t c = b_ci[f];\n                if (!seen[c]) {\n                    seen[c] = 1;\n                    list[cnt++] = c;",
     "                int32_t c = b_ci[f];\n                if (f == b_ro[j] && j == 0) continue;\n                if (!seen[c]) {\n                    seen[c] = 1;\n                    list[cnt++] = c;"),
    ("spgemm_unsorted", "        qsort(cols, (size_t)cnt, sizeof *cols, orc_cmp_i32);", "        (void)orc_cmp_i32;"),
    ("bf16_shift", "uint32_t bits = (uint32_t)((const uint16_t *)p)[i] << 16;", "uint32_t bits = (uint32_t)((const uint16_t *)p)[i] << 15;"),
]


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    return tmp_path_factory.mktemp("mutants")


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, mutant_dir):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new, 1)
    path = mutant_dir / f"{name}.c"
    path.write_text(mutated)
    so = str(mutant_dir / f"lib{name}.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", str(path), "-o", so], check=True)
    orc = oracle.Oracle(so)
    caught = []
    for pin in ALL_PINS:
        try:
            pin(orc)
        except (AssertionError, ValueError, IndexError):
            caught.append(pin.__name__)
    assert caught, f"no pin catches the planted mistake {name}"
