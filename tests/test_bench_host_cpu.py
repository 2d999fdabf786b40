"""Host logic of bench.py: the kernel-source hash that decides whether the
committed counter profile still describes the measured kernels, and the
algorithmic byte count the roofline divides by."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_of_drops_comments_and_blank_lines():
    src = ('int a = 1;   // trailing note\n'
           '/* a block\n   comment */\n'
           '\n'
           'const char *s = "x // y /* z */";\n'
           "char q = '\"';  // a quote in a character literal\n"
           'int b = 2; /* inline */ int c = 3;\n')
    assert bench._code_of(src) == ('int a = 1;\n'
                                   'const char *s = "x // y /* z */";\n'
                                   "char q = '\"';\n"
                                   'int b = 2;   int c = 3;')


def test_code_of_keeps_escaped_quotes_inside_literals():
    src = 'const char *s = "a \\" // not a comment";\nint x;  // gone\n'
    assert bench._code_of(src) == 'const char *s = "a \\" // not a comment";\nint x;'


def test_comment_edits_keep_the_hash_code_edits_change_it():
    base = '__device__ int f(int x)\n{\n    return x + 1;   // one more\n}\n'
    comment_only = '// what f does\n__device__ int f(int x)\n{\n\n    return x + 1;\n}\n'
    code_edit = '__device__ int f(int x)\n{\n    return x + 2;   // one more\n}\n'
    assert bench._code_of(base) == bench._code_of(comment_only)
    assert bench._code_of(base) != bench._code_of(code_edit)


def test_kernel_source_hash_is_stable_and_short():
    h = bench.kernel_source_hash()
    assert h == bench.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)


def test_algorithmic_bytes_terms():
    # one voxel update: read + write of (distance, weight) in binary32
    assert bench.algorithmic_bytes(1, 0, 0, 0, 0) == 16
    # binary16 storage halves the voxel term
    assert bench.algorithmic_bytes(1, 0, 0, 0, 0, voxel_bytes=4) == 8
    # a 640x480 frame's depth pixels, read once each
    assert bench.algorithmic_bytes(0, 0, 0, 640 * 480, 1) == 4 * 640 * 480
    # touched block: key and value read + list entry; new block: key, value, slot key
    assert bench.algorithmic_bytes(0, 1, 0, 0, 0) == 16
    assert bench.algorithmic_bytes(0, 0, 1, 0, 0) == 20
