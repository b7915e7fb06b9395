"""The kernel-code hash that keeps a committed HBM-traffic figure tied to the
code it was measured on: comment, blank-line and indentation edits keep it,
any code edit changes it, and the traffic reader refuses a summary whose hash
is not the current one."""
import hashlib
import os

from paper_2005_11547_amd import profiling as P


def _hash_of(texts):
    h = hashlib.sha256()
    for t in texts:
        h.update(P.code_text(t).encode())
    return h.hexdigest()[:16]


def _sources():
    return [open(os.path.join(P.HERE, f), encoding="utf-8").read() for f in P.KERNEL_SOURCES]


def test_hash_matches_the_sources():
    assert P.source_hash() == _hash_of(_sources())


def test_comment_and_layout_edits_keep_the_hash():
    src = _sources()
    edited = ["// a new comment line\n\n" + t.replace("\n", "\n\n", 3) for t in src]
    edited[0] = edited[0].replace("namespace dms {", "namespace dms {  // trailing comment", 1)
    assert _hash_of(edited) == _hash_of(src)


def test_code_edits_change_the_hash():
    src = _sources()
    changed = list(src)
    changed[0] = changed[0].replace("constexpr int kLowLevels = 3;", "constexpr int kLowLevels = 2;", 1)
    assert changed[0] != src[0]
    assert _hash_of(changed) != _hash_of(src)


def test_code_text_strips_comments_blank_lines_and_indentation():
    text = "int a = 1;  // one\n\n    // only a comment\n\tint b = 2;\n"
    assert P.code_text(text) == "int a = 1;\nint b = 2;"


def test_traffic_reader_requires_the_current_hash(tmp_path):
    good = tmp_path / "good.txt"
    good.write_text(f"traffic_bytes: 12345\nsource_hash: {P.source_hash()}\n")
    stale = tmp_path / "stale.txt"
    stale.write_text("traffic_bytes: 12345\nsource_hash: 0000000000000000\n")
    assert P.read_traffic(str(good)) == 12345.0
    assert P.read_traffic(str(stale)) is None
    assert P.read_traffic(str(tmp_path / "missing.txt")) is None
