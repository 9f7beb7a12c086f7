"""Host-side checks of the profiling helpers (CPU): the source hash that ties
a committed counter summary to the code it was taken on follows the code,
not its comments or layout."""
import os

from paper_1306_4161_amd import profiling


def test_code_only_drops_comments_and_keeps_literals():
    src = ('int a = 1;  // trailing\n'
           '/* a block\n   comment */ const char* s = "x // y /* z */";\n'
           "char q = '\\''; char r = '/';\n\n\tint   b;")
    assert profiling.code_only(src) == (
        'int a = 1; const char* s = "x // y /* z */"; '
        "char q = '\\''; char r = '/'; int b;")
    # a comment edit or a reflow leaves the code unchanged; a code edit does not
    assert profiling.code_only("x = 1; // one") == profiling.code_only("x  =  1;  // two")
    assert profiling.code_only("x = 1;") != profiling.code_only("x = 2;")


def test_committed_summaries_match_the_current_code():
    # every counter summary under profiles/ names the hash of the sources it
    # was taken on; bench.py reports its traffic only while they agree
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    prof = os.path.join(root, "profiles")
    seen = 0
    for name in sorted(os.listdir(prof)):
        if not (name.startswith("traffic_") or name.startswith("mfma_busy_")):
            continue
        text = open(os.path.join(prof, name)).read()
        cmd = [ln for ln in text.splitlines() if "--source" in ln][0]
        srcs = cmd.split("--source", 1)[1].split()[0]
        got = [ln.split(":", 1)[1].strip() for ln in text.splitlines()
               if ln.startswith("source_hash:")][0]
        assert got == profiling.source_hash(*srcs.split(",")), name
        seen += 1
    assert seen >= 8
