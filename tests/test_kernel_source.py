"""Static checks of the HIP source (CPU): the buffer-resource accessors, which address GLOBAL
memory through a scalar descriptor, must never be handed an LDS vector.  (An LDS address used as
a global buffer base is a wild global access.)"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2511_17634_amd", "csrc", "xkp_kernels.hip")
GLOBAL_ONLY = ("load_rows", "store_rows", "load_col", "store_col", "mkbuf", "mkbuf32",
               "mkbuf16", "load_buf", "load_buf_f32", "store_col_f32", "store_col_bf16",
               "load_col_any", "sweep_cols")
LDS_NAMES = re.compile(r"^\s*(vbuf|lds|Ap|zv|alpha|red|L\.\w+)\b")


def calls(src, fn):
    for m in re.finditer(r"\b%s(?:<[^>]*>)?\(" % fn, src):
        yield src[m.end():m.end() + 80], src.count("\n", 0, m.start()) + 1


def test_no_lds_pointer_reaches_a_buffer_accessor():
    src = open(SRC).read()
    bad = []
    for fn in GLOBAL_ONLY:
        for arg, line in calls(src, fn):
            if LDS_NAMES.match(arg):
                bad.append(f"{fn}({arg.split(',')[0]}) at line {line}")
    assert not bad, bad


def test_lds_stores_use_the_lds_helper():
    src = open(SRC).read()
    assert "store_rows_lds<RMAX>(vbuf" in src or "store_rows_lds<RMAX>(L.vbuf" in src
