"""The profile summaries' source hash ignores comments and layout but not code."""
from paper_2009_07226_amd import pmc_summary as p


def test_code_only_drops_comments_keeps_literals():
    a = 'int a = 1; // note\n/* block\n comment */ const char *s = "// not a comment";\nchar c = \'/\';'
    b = 'int a = 1;\n  const char *s = "// not a comment"; char c = \'/\'; // other note'
    assert p.code_only(a) == p.code_only(b)
    assert "not a comment" in p.code_only(a)
    assert p.code_only("x = 1;") != p.code_only("x = 2;")


def test_kernel_sources_sha_is_stable():
    assert p.kernel_sources_sha() == p.kernel_sources_sha()
    assert len(p.kernel_sources_sha()) == 64
