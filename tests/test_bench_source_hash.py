"""The bench reports a precision's counter summaries only while its kernel sources hash to the value
recorded with them; the hash covers the code with comments removed and whitespace collapsed (CPU only)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_code_tokens_drop_comments_and_layout_only():
    src = ('int a = 1;  // trailing "quoted"\n/* block\n   comment */ const char *s = "x // y /* z */";\n'
           "char c = '/';\n\tb  =  a;\n")
    assert bench.code_tokens(src) == "int a = 1; const char *s = \"x // y /* z */\"; char c = '/'; b = a;"
    # a comment edit or a re-indent keeps the tokens; a code edit changes them
    assert bench.code_tokens(src.replace("trailing", "other")) == bench.code_tokens(src)
    assert bench.code_tokens(src.replace("\tb  =  a;", "b = a;")) == bench.code_tokens(src)
    assert bench.code_tokens(src.replace("b  =  a", "b = a + 1")) != bench.code_tokens(src)

