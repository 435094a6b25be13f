"""Shared cases of the regular-expression tests: expressions in the front-end's
syntax with their Python equivalents, and the brute-force reference."""
import re


def brute(py: str, s: bytes, mode: str):
    """(accept, count) from Python's re: anchored counts prefixes in the
    language, search counts the ends of matches."""
    pat = re.compile(py.encode(), re.S)
    if mode == "anchored":
        count = sum(1 for i in range(len(s)) if pat.fullmatch(s[:i + 1]))
        return bool(pat.fullmatch(s)), count
    count = sum(1 for i in range(len(s)) if any(pat.fullmatch(s[j:i + 1]) for j in range(i + 2)))
    return any(pat.fullmatch(s[j:]) for j in range(len(s) + 1)), count


def dfa_run(table, fin, s: bytes, alphabet: bytes):
    """Walk the front-end's table from state 0 (test-side: the definition of
    a DFA run); (accept, count, died)."""
    col = {c: j for j, c in enumerate(alphabet)}
    q, count = 0, 0
    for x in s:
        q = int(table[q, col[x]])
        if q == 0xFFFFFFFF:
            return False, count, True
        count += int(fin[q])
    return bool(fin[q]), count, False


# (ours, Python's) - the same language; postfix operators bind tighter than
# concatenation, which binds tighter than union, in both
FIXED = [
    (b"(a|b)?c*[0..3]b+", "(a|b)?c*[0-3]b+", b"abc0123"),
    (b"a|b*", "a|b*", b"ab"),
    (b"(a|b)*", "(a|b)*", b"ab"),
    (b"(ab|c)*", "(ab|c)*", b"abc"),
    (b"ab|c", "ab|c", b"abc"),
    (b"a(b|c)d", "a(b|c)d", b"abcd"),
    (b"ab+", "ab+", b"ab"),
    (b"(ab)+", "(ab)+", b"ab"),
    (b"a?b?", "a?b?", b"ab"),
    (b"(|a)b", "(|a)b", b"ab"),
    (b"a(b+)?", "a(?:b+)?", b"ab"),
    (b"[a..c]+x", "[a-c]+x", b"abcx"),
    (b"[ab-c]x|y", "[ab-c]x|y", b"abcxy"),
    (b"\\*a|\\(", "\\*a|\\(", b"a*("),
    (b"", "", b"ab"),
    (b"()", "()", b"ab"),
    (b"parallel", "parallel", b"parel"),
]


def random_expression(rng, alpha: bytes, depth: int):
    """A random expression in both syntaxes (ours, Python's)."""
    k = int(rng.integers(0, 7 if depth > 0 else 2))
    if k == 0:
        c = bytes([alpha[int(rng.integers(0, len(alpha)))]])
        return c, re.escape(c.decode())
    if k == 1:
        lo, hi = sorted(rng.choice(sorted(alpha), size=2))
        return b"[" + bytes([lo]) + b".." + bytes([hi]) + b"]", f"[{re.escape(chr(lo))}-{re.escape(chr(hi))}]"
    a, pa = random_expression(rng, alpha, depth - 1)
    if k in (2, 3):
        b, pb = random_expression(rng, alpha, depth - 1)
        if k == 2:
            return a + b, pa + pb
        return b"(" + a + b"|" + b + b")", f"(?:{pa}|{pb})"
    op = {4: b"*", 5: b"+", 6: b"?"}[k]
    return b"(" + a + b")" + op, f"(?:{pa}){op.decode()}"
