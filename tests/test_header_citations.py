"""Every entry point of include/qsv.h documents the passage of the paper
that defines its operation (a Section, Table or equation), except the
control calls and the one allocation-free variant, whose comments say
so."""
import os
import re

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include",
                      "qsv.h")
CITE = re.compile(r"Sections? [IV]+(\.[A-Z])?|Table [IV]+|eqs? \d")


def declarations():
    """(name, comment) for each function declaration: the comment is the
    /* ... */ block that precedes it (shared by declarations that follow one
    comment directly)."""
    text = open(HEADER).read()
    out = []
    last_comment = ""
    token = re.compile(r"/\*.*?\*/|^(?:qsv_status|const char\*|double)\s+"
                       r"(qsv_\w+)\s*\(", re.S | re.M)
    for m in token.finditer(text):
        if m.group(0).startswith("/*"):
            # one line of text: drop the " * " prefixes of continued lines
            last_comment = " ".join(
                ln.strip().lstrip("*").strip()
                for ln in m.group(0).splitlines())
        else:
            out.append((m.group(1), last_comment))
    return out


def test_every_entry_point_cites_its_passage_or_is_a_control_call():
    decls = declarations()
    assert len(decls) >= 40
    missing = [name for name, c in decls
               if not CITE.search(c) and "(Control call.)" not in c
               and "(For callers that cannot allocate.)" not in c]
    assert not missing, missing


def test_one_allocation_free_variant():
    noalloc = [name for name, c in declarations()
               if "(For callers that cannot allocate.)" in c]
    assert noalloc == ["qsv_renormalize_noalloc"]


def test_control_calls_are_few():
    control = [name for name, c in declarations()
               if "(Control call.)" in c and not CITE.search(c)]
    assert len(control) <= 16, control
