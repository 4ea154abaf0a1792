"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

Every check here is independent of the oracle's own code: worked-example
values printed in arXiv 2503.06763 (tests/golden/*.yaml, each citing its
source), a brute-force tree enumerator with its own RE reader
(tests/lst_brute.py), Python's ``re`` module for acceptance, closed forms, and
invariants of the SLPF.
"""
import itertools
import os
import re

import numpy as np
import pytest
import yaml

import lst_brute
from automata_props import column_unambiguous
from gen import regen
from oracle.oracle import P61, Oracle, OracleError, STATUS_INF_AMBIG, STATUS_SYNTAX

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name), encoding="utf-8") as f:
        return yaml.safe_load(f)


# ------------------------------------------------------------ e2 (Sect. 2-3)

@pytest.fixture(scope="module")
def e2():
    g = load("e2.yaml")
    o = Oracle(g["re"])
    # paper number -> oracle id, through the segment strings
    pid = {int(k): o.seg_id(v) for k, v in g["segments"].items()}
    return g, o, pid


def _ids(pid, nums):
    return frozenset(pid[int(x)] for x in nums)


def test_e2_segments(e2):
    g, o, pid = e2
    assert sorted(o.segments) == sorted(g["segments"].values())
    assert o.I == _ids(pid, g["initial"])
    assert o.F == _ids(pid, g["final"])


def test_e2_folseg(e2):
    g, o, pid = e2
    for p, fol in g["folseg"].items():
        assert o.folseg[pid[int(p)]] == _ids(pid, fol), p


def _check_automaton(o, pid, states, trans, gold):
    named = {name: _ids(pid, segs) for name, segs in gold["states"].items()}
    assert sorted(map(sorted, states)) == sorted(map(sorted, named.values()))
    idx = {s: i for i, s in enumerate(states)}
    for letter in "ab":
        a = ord(letter)
        expect = gold["delta"].get(letter, {})
        for name, s in named.items():
            t = trans[(idx[s], a)]
            got = states[t] if t is not None else None
            want = named[expect[name]] if name in expect else None
            assert got == want, (letter, name)


def test_e2_dfa(e2):
    g, o, pid = e2
    states, trans = o.dfa([ord("a"), ord("b")])
    _check_automaton(o, pid, states, trans, g["dfa"])


def test_e2_medfa(e2):
    g, o, pid = e2
    states, trans = o.medfa([ord("a"), ord("b")])
    _check_automaton(o, pid, states, trans, g["medfa"])


def test_e2_ex4_serial(e2):
    g, o, pid = e2
    ex = g["ex4"]
    x = ex["text"].encode()
    # forward and backward columns of Eq. matrixmul, one step at a time
    fwd = [o.I]
    for a in x:
        fwd.append(o.step_fwd(fwd[-1], a))
    bwd = [o.F]
    for a in reversed(x):
        bwd.append(o.step_bwd(bwd[-1], a))
    bwd.reverse()
    assert fwd == [_ids(pid, c) for c in ex["forward"]]
    assert bwd == [_ids(pid, c) for c in ex["backward"]]
    cols, acc, cnt = o.columns(x)
    assert cols == [_ids(pid, c) for c in ex["clean"]]
    assert acc and cnt == 1


def test_e2_ex6_parallel(e2):
    g, o, pid = e2
    ex = g["ex6"]
    tr = o.parallel_trace(ex["text"].encode(), ex["k"])
    want_R = {tuple(map(int, k.split(","))): v for k, v in ex["R"].items()}
    for (i, j), s in tr["R"].items():
        paper_j = [p for p, q in pid.items() if q == j][0]
        want = _ids(pid, want_R.get((i, paper_j), []))
        assert s == want, (i, paper_j)
    assert tr["J"] == [_ids(pid, c) for c in ex["J"]]
    assert [tr["B"][r] for r in range(1, 7)] == [_ids(pid, c) for c in ex["B"]]
    assert [tr["Bh"][r] for r in range(1, 7)] == [_ids(pid, c) for c in ex["Bh"]]
    assert tr["C"] == [_ids(pid, c) for c in ex["C"]]
    cols, acc, cnt = o.columns(ex["text"])
    assert cols == tr["C"] and acc and cnt == ex["trees"]


def test_e2_compact_encoding(e2):
    # hand-derived candidate lists and compact words of Ex. 6 (App. SLPF
    # optimization); the order inside a list is the segment order of Tab.
    # segments, which the canonical order keeps for e2's lists
    g, o, pid = e2
    byte = {"start": None, "end": None, "a": ord("a"), "b": ord("b")}
    for key, want in g["candidates"].items():
        p, q = key.split(",")
        got = o.candidates(byte[p], byte[q])
        assert got == [pid[k] for k in want], key
    ex = g["ex6"]
    assert o.compact(ex["text"].encode()).tolist() == g["compact_ex6"]


def _decode_compact(o, x, words):
    out = []
    for r, w in enumerate(words.tolist()):
        cand = o.candidates(x[r - 1] if r > 0 else None, x[r] if r < len(x) else None)
        out.append(frozenset(cand[k] for k in range(64) if (w >> k) & 1))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_compact_is_lossless_and_columns_lie_in_candidates(seed):
    # every clean column lies inside its candidate list (the invariant the
    # encoding rests on) and decoding the words gives the columns back
    tree = regen.random_re(900 + seed, n_ops=10, max_depth=5, alphabet=b"abc")
    o = Oracle(regen.to_re(tree))
    rng = np.random.default_rng(seed)
    from gen import textgen
    for j in range(4):
        t = textgen.sample_text(tree, seed * 10 + j, int(rng.integers(0, 300))).tobytes()
        cols, acc, _ = o.parse(t)
        words = o.compact(t, cols)
        assert _decode_compact(o, t, words) == [o.to_set(c) for c in cols]
        assert all(w != 0 for w in words.tolist()) == acc


def _brute_matches(re_, text, g):
    """Group spans over every LST (brute force): "g(" at position p and its
    matching ")g" at position q, positions counted in terminals."""
    o, c = "%d(" % g, ")%d" % g
    out = set()
    for t in lst_brute.lsts(re_, text):
        p, stack = 0, []
        for tok in t:
            if tok == o:
                stack.append(p)
            elif tok == c:
                out.add((stack.pop(), p))
            elif lst_brute.is_end_letter(tok):
                p += 1
    return sorted(out)


MATCH_CASES = [
    ("(ab|a)*", [b"", b"a", b"ab", b"abaaba", b"aab"]),
    ("(a|b|ab)+", [b"abab", b"a", b"bab"]),
    ("(a|ab|aba)+", [b"aba", b"abaab"]),
    ("(a|())b", [b"b", b"ab"]),
    ("((a|b)*c)+", [b"abcbc", b"c", b"cc"]),
    ("(a?b)*(ab?)*", [b"abab", b"aab", b"ba"]),
    ("x(y|yz)*(z|zy)*", [b"xyzzy", b"xyzyz"]),
]


@pytest.mark.parametrize("re_,texts", MATCH_CASES)
def test_match_extraction_equals_brute_force(re_, texts):
    # every group's match set equals the spans over all enumerated trees
    o = Oracle(re_)
    groups = sorted({int(t[:-1]) for seg in o.segments for t in seg.split(" ") if t.endswith("(")})
    for text in texts:
        for g in groups:
            assert o.matches(text, g) == _brute_matches(re_.encode(), text, g), (re_, text, g)


def test_match_extraction_rejected_and_e2_example():
    o = Oracle("(ab|a)*")
    assert o.matches(b"abb", 1) == [] and o.matches(b"b", 2) == []
    # Ex. 6, "abaaba" = (ab)(a)(ab)(a): the union group 2 spans each factor,
    # the concatenation 3 the two "ab", the star 1 the whole text
    assert o.matches(b"abaaba", 2) == [(0, 2), (2, 3), (3, 5), (5, 6)]
    assert o.matches(b"abaaba", 3) == [(0, 2), (3, 5)]
    assert o.matches(b"abaaba", 1) == [(0, 6)]


def _brute_children(re_, text, g, start, end):
    """The direct children of g's occurrences over (start, end), over every
    LST (brute force): each subtree directly inside such an occurrence, as
    (node, a, b); a terminal spans one byte, an epsilon none."""
    out = set()
    for t in lst_brute.lsts(re_, text):
        p, stack = 0, []                 # open subtrees: [node, start, children]
        for tok in t:
            if tok.endswith("("):
                stack.append([int(tok[:-1]), p, []])
                continue
            if tok.startswith(")"):
                k, a, kids = stack.pop()
                b = p
                if k == g and (a, b) == (start, end):
                    out.update(kids)
            else:
                k, a = lst_brute.leaf_number(tok), p
                b = p + 1 if lst_brute.is_end_letter(tok) else p
                p = b
            if stack:
                stack[-1][2].append((k, a, b))
    return sorted(out)


def _check_children(o, re_, text, n_groups):
    cols = o.parse(text)[0]
    n = len(text)
    for g in range(1, n_groups + 1):
        spans = set(_brute_matches(re_, text, g))
        # every match of g, and some spans that are not matches
        probe = spans | {(0, n), (n // 2, n), (0, n // 2), (n, n)}
        for (a, b) in sorted(probe):
            want = _brute_children(re_, text, g, a, b) if (a, b) in spans else []
            assert o.children(text, g, a, b, cols=cols) == want, (re_, text, g, a, b)


@pytest.mark.parametrize("re_,texts", MATCH_CASES)
def test_children_equal_brute_force(re_, texts):
    # getChildren: the children of every match of every node equal the
    # subtrees directly inside that node's occurrences over all trees
    o = Oracle(re_)
    for text in texts:
        _check_children(o, re_.encode(), text, o.num_nodes)


@pytest.mark.parametrize("seed", range(12))
def test_children_equal_brute_force_random(seed):
    rng = np.random.default_rng(3000 + seed)
    pat = regen.to_re(_tiny_random_re(rng))
    o = Oracle(pat)
    for x in _strings("ab", 4):
        _check_children(o, pat, x, o.num_nodes)


def test_children_e2_example():
    # Ex. 6 tree of "abaaba": the star's children are the four factors, the
    # union's child over "ab" the concatenation, whose children are a and b
    o = Oracle("(ab|a)*")
    assert o.children(b"abaaba", 1, 0, 6) == [(2, 0, 2), (2, 2, 3), (2, 3, 5), (2, 5, 6)]
    assert o.children(b"abaaba", 2, 0, 2) == [(3, 0, 2)]
    assert o.children(b"abaaba", 2, 2, 3) == [(6, 2, 3)]
    assert o.children(b"abaaba", 3, 3, 5) == [(4, 3, 4), (5, 4, 5)]
    assert o.children(b"abaaba", 1, 0, 5) == [] and o.children(b"abaaba", 4, 0, 1) == []


# ------------------------------------------------------------ e3, e1, e4

def test_e3_nfa_and_slpf():
    g = load("e3.yaml")
    o = Oracle(g["re"])
    assert sorted(o.segments) == sorted(g["segments"])
    cols, acc, cnt = o.columns(b"abab")
    got = [sorted(o.segments[i] for i in c) for c in cols]
    assert got == [sorted(c) for c in g["abab"]["columns"]]
    assert acc and cnt == len(g["abab"]["trees"]) == 4
    assert sorted(" ".join(t) for t in lst_brute.lsts(g["re"].encode(), b"abab")) == sorted(g["abab"]["trees"])


def test_e1_two_trees():
    g = load("e1_e4.yaml")["e1"]
    o = Oracle(g["re"])
    cols, acc, cnt = o.columns(g["text"])
    assert acc and cnt == 2
    trees = lst_brute.lsts(g["re"].encode(), g["text"].encode())
    assert sorted(" ".join(t) for t in trees) == sorted(g["trees"])


def test_e4_epsilon_in_meta_prefix():
    g = load("e1_e4.yaml")["e4"]
    o = Oracle(g["re"])
    cols, acc, cnt = o.columns(g["text"])
    assert acc and cnt == 1
    assert [o.segments[min(c)] for c in cols] == g["path"]
    assert [" ".join(t) for t in lst_brute.lsts(g["re"].encode(), g["text"].encode())] == g["trees"]


def test_ek_dfa_state_count():
    g = load("ek_statecount.yaml")
    for k, want in zip(g["k"], g["dfa_states"]):
        o = Oracle("(a|b)*a" + "(a|b)" * k)
        states, _ = o.dfa()
        assert len(states) == want == 2 ** (k + 1) + 1
        # the ME-DFA has one entry per segment: linear in k
        assert o.nseg == 2 * k + 7


# ------------------------------------------------------------ brute force

def _tiny_random_re(rng):
    """Random tree, depth <= 3, <= 6 operators, over {a, b, c} with epsilon."""
    def leaf():
        r = rng.random()
        if r < 0.1:
            return regen.EPS
        return regen.lit("abc"[int(rng.integers(3))])

    def grow(d, budget):
        if d >= 3 or budget[0] <= 0 or rng.random() < 0.3:
            return leaf()
        budget[0] -= 1
        k = ["cat", "alt", "star", "plus", "opt"][int(rng.integers(5))]
        if k in ("cat", "alt"):
            return (k, [grow(d + 1, budget) for _ in range(int(rng.integers(2, 4)))])
        return (k, grow(d + 1, budget))
    while True:
        t = grow(0, [6])
        if t[0] not in ("lit", "eps") and not regen.infinitely_ambiguous(t):
            return t


def _strings(alpha, maxlen):
    for n in range(maxlen + 1):
        for t in itertools.product(alpha, repeat=n):
            yield "".join(t).encode()


@pytest.mark.parametrize("seed", range(40))
def test_oracle_equals_brute_force(seed):
    rng = np.random.default_rng(1000 + seed)
    tree = _tiny_random_re(rng)
    pat = regen.to_re(tree)
    o = Oracle(pat)
    py = re.compile(pat.decode())
    for x in _strings("abc", 5):
        cols, acc, cnt = o.columns(x)
        bcols, bcnt = lst_brute.clean_columns(pat, x)
        assert [set(o.segments[i] for i in c) for c in cols] == bcols, (pat, x)
        assert cnt == bcnt, (pat, x)
        assert o.parse_full(x)[3] == bcnt % P61, (pat, x)
        assert acc == (bcnt > 0) == (py.fullmatch(x.decode()) is not None), (pat, x)


def test_brute_force_on_listed_res():
    for pat in [b"(a|ab|b)*(c|bc)+(a|b)*", b"(a|b|ab)+", b"(ab|a)*", b"a(bc)", b"(a?b?)c",
                b"((a|b)(c|()))+", b"(a*|b*)c", b"a|()", b"()"]:
        o = Oracle(pat)
        for x in _strings("abc", 5):
            cols, acc, cnt = o.columns(x)
            bcols, bcnt = lst_brute.clean_columns(pat, x)
            assert [set(o.segments[i] for i in c) for c in cols] == bcols, (pat, x)
            assert cnt == bcnt, (pat, x)


# ------------------------------------------------------------ closed forms

@pytest.mark.parametrize("pat", ["(a|ab|b)*", "(a|b|ab)+"])
def test_count_is_two_to_the_ab_occurrences(pat):
    o = Oracle(pat)
    rng = np.random.default_rng(5)
    for _ in range(60):
        n = int(rng.integers(1, 40))
        x = bytes(rng.choice([97, 98], size=n).tolist())
        _, acc, cnt, cntp = o.parse_full(x)
        assert acc and cnt == (2 ** x.count(b"ab")) % (1 << 64)
        assert cntp == pow(2, x.count(b"ab"), P61)
    x = b"ab" * 70                      # 2^70 wraps to 0 modulo 2^64, to 2^9 modulo 2^61 - 1
    _, acc, cnt, cntp = o.parse_full(x)
    assert acc and cnt == 0 and cntp == 512
    x = b"ab" * 63 + b"a"
    _, acc, cnt, cntp = o.parse_full(x)
    assert acc and cnt == 2 ** 63 and cntp == 4


def _fib(n):
    a, b = 0, 1
    for _ in range(n):
        a, b = b, a + b
    return a


def test_count_closed_forms_both_moduli():
    # (a|aa)* over a^n: the compositions of n into parts 1 and 2, F(n+1);
    # ten equal alternatives under a star over a^n: 10^n.  Exact integers
    # reduced modulo 2^64 and modulo 2^61 - 1 (sums past both moduli)
    o = Oracle("(a|aa)*")
    for n in (0, 1, 2, 3, 10, 92, 93, 94, 150, 300):
        _, acc, cnt, cntp = o.parse_full(b"a" * n)
        want = _fib(n + 1)
        assert acc and cnt == want % (1 << 64) and cntp == want % P61, n
    o = Oracle("(a|a|a|a|a|a|a|a|a|a)*")
    for n in (0, 1, 5, 19, 20, 64, 100):
        _, acc, cnt, cntp = o.parse_full(b"a" * n)
        assert acc and cnt == pow(10, n, 1 << 64) and cntp == pow(10, n, P61), n
    # rejected text: both counts zero
    _, acc, cnt, cntp = o.parse_full(b"ab")
    assert not acc and cnt == 0 and cntp == 0


def test_unambiguous_counts_are_zero_or_one():
    for pat in ["(ab|a)*", "(a|b)*a(a|b)(a|b)"]:
        o = Oracle(pat)
        for x in _strings("ab", 8):
            _, acc, cnt = o.columns(x)
            assert cnt == int(acc)


@pytest.mark.parametrize("seed", range(40))
def test_column_unambiguous_res_have_one_tree(seed):
    # the fact behind the count's shortcut for such REs: when no reachable
    # forward and reverse state sets share two segments, the brute-force
    # enumerator finds at most one tree for every text, and the clean columns
    # are single segments
    rng = np.random.default_rng(5000 + seed)
    tree = _tiny_random_re(rng)
    pat = regen.to_re(tree)
    o = Oracle(pat)
    if not column_unambiguous(o):
        pytest.skip("RE not column-unambiguous")
    for x in _strings("abc", 5):
        bcols, bcnt = lst_brute.clean_columns(pat, x)
        assert bcnt <= 1, (pat, x)
        assert all(len(c) <= 1 for c in bcols), (pat, x)


def test_column_unambiguity_is_not_vacuous():
    # the property holds for some of the random REs above and fails for
    # ambiguous ones
    hits = sum(column_unambiguous(Oracle(regen.to_re(_tiny_random_re(np.random.default_rng(5000 + s)))))
               for s in range(40))
    assert 5 <= hits < 40
    for pat in ["(a|ab|b)*", "(a|aa)*", "(a|b|ab)+"]:
        assert not column_unambiguous(Oracle(pat))
    for pat in ["(ab|cd)*e", "x(yz)*", "(ab|a)*"]:
        assert column_unambiguous(Oracle(pat))


# ------------------------------------------------------------ invariants

@pytest.mark.parametrize("seed", range(6))
def test_slpf_invariants(seed):
    rng = np.random.default_rng(77 + seed)
    tree = regen.random_re(seed, n_ops=12, max_depth=4, alphabet=b"abcd")
    pat = regen.to_re(tree)
    o = Oracle(pat)
    from gen import textgen
    for t in range(4):
        x = textgen.sample_text(tree, 100 * seed + t, int(rng.integers(0, 300))).tobytes()
        if t == 3 and x:
            x = x[:-1] + b"z"          # a byte outside the alphabet: rejected, not an error
        cols, acc, cnt = o.columns(x)
        nonempty = [bool(c) for c in cols]
        assert all(nonempty) == acc and (any(nonempty) == acc)
        if acc:
            assert cols[0] <= o.I and cols[-1] <= o.F
            for r in range(len(x)):
                assert all(x[r] in o.label_sets[s] for s in cols[r])
        else:
            assert cnt == 0
        if t < 3:
            assert acc, "sampled texts are in the language"


@pytest.mark.parametrize("seed", range(8))
def test_dfa_parser_equals_nfa_parser(seed):
    tree = regen.random_re(50 + seed, n_ops=15, max_depth=5, alphabet=b"abc")
    pat = regen.to_re(tree)
    o = Oracle(pat)
    from gen import textgen
    x = textgen.sample_text(tree, seed, 2000).tobytes()
    if seed % 2:
        x = x[:len(x) // 2] + b"c" + x[len(x) // 2:]
    cols, acc, cnt, cntp = o.parse_full(x)
    n = len(x)
    starts = [0, n // 3, max(n - 50, 0)]
    win, acc2, cnt2, cntp2 = o.parse_dfa_full(x, starts, 50)
    assert acc == acc2 and cnt == cnt2 and cntp == cntp2
    for i, s in enumerate(starts):
        m = min(50, n + 1 - s)
        assert np.array_equal(win[i, :m], cols[s:s + m])


def test_parallel_trace_matches_serial_for_all_chunkings():
    """Eq. reacher/joiner/builder/merger reproduce the serial SLPF for any k."""
    o = Oracle("(a|ab|b)*(c|bc)+(a|b)*")
    x = b"abbabcbcbccab"
    cols = o.columns(x)[0]
    for k in range(1, len(x) + 1):
        tr = o.parallel_trace(x, k)
        assert tr["C"] == cols, k
        c = len(tr["J"]) - 1
        for i in range(1, c + 1):          # M at a chunk edge is J_i cap Jh_{i+1}
            r = min(i * k, len(x))
            assert tr["M"][r] == tr["J"][i] & tr["Jh"][i + 1]


# ------------------------------------------------------------ errors

def test_rejects():
    with pytest.raises(OracleError) as e:
        Oracle("(a|b")
    assert e.value.status == STATUS_SYNTAX
    with pytest.raises(OracleError) as e:
        Oracle("a)")
    assert e.value.status == STATUS_SYNTAX
    with pytest.raises(OracleError) as e:
        Oracle("*a")
    assert e.value.status == STATUS_SYNTAX
    # App. A, infinitely ambiguous RE: an iterator over a nullable body
    for pat in ["(a|())*", "(a*)*", "(a?b?)+", "(()|b*)+"]:
        with pytest.raises(OracleError) as e:
            Oracle(pat)
        assert e.value.status == STATUS_INF_AMBIG, pat


def test_empty_text():
    o = Oracle("(ab|a)*")
    cols, acc, cnt = o.columns(b"")
    assert acc and cnt == 1 and cols == [o.I & o.F]
    o = Oracle("a(b|c)")
    cols, acc, cnt = o.columns(b"")
    assert not acc and cnt == 0 and cols == [frozenset()]


# ------------------------------------------- character sets and the wildcard

_SET_LEAVES = [b"[ab]", b"[a-c]", b"[^a]", b".", b"[bc]", b"[ac]", b"a", b"b", b"c"]


def _tiny_set_re(rng):
    """A tiny RE over {a, b, c} whose leaves are bytes, character sets or the
    wildcard (App. A, character features), not infinitely ambiguous."""
    def grow(d, budget):
        if d >= 3 or budget[0] <= 0 or rng.random() < 0.3:
            return _SET_LEAVES[int(rng.integers(len(_SET_LEAVES)))]
        budget[0] -= 1
        k = int(rng.integers(5))
        if k < 2:
            parts = [grow(d + 1, budget) for _ in range(int(rng.integers(2, 4)))]
            return b"(" + (b"" if k == 0 else b"|").join(parts) + b")"
        return b"(" + grow(d + 1, budget) + b")" + b"*+?"[k - 2:k - 1]
    while True:
        pat = grow(0, [6])
        try:
            Oracle(pat)
            return pat
        except OracleError as e:
            assert e.status == STATUS_INF_AMBIG


@pytest.mark.parametrize("seed", range(30))
def test_char_sets_equal_brute_force_and_re(seed):
    # columns and counts against the brute-force LST enumerator (its own RE
    # reader), accept against Python's re (same bracket and dot syntax)
    rng = np.random.default_rng(7000 + seed)
    pat = _tiny_set_re(rng)
    o = Oracle(pat)
    py = re.compile(pat)
    for x in _strings("abc", 5):
        cols, acc, cnt = o.columns(x)
        bcols, bcnt = lst_brute.clean_columns(pat, x)
        assert [set(o.segments[i] for i in c) for c in cols] == bcols, (pat, x)
        assert cnt == bcnt and o.parse_full(x)[3] == bcnt, (pat, x)
        assert acc == (bcnt > 0) == (py.fullmatch(x) is not None), (pat, x)


def _expand_sets(pat: bytes) -> bytes:
    """The same RE with every set and wildcard written as a union of single
    bytes over a b c and the newline (only those occur in the texts below)."""
    out, k = b"", 0
    universe = b"abc\n"
    while k < len(pat):
        c = pat[k:k + 1]
        if c == b"[":
            e = pat.index(b"]", k + 2)
            members = set(re.findall(rb".", pat[k:e + 1]) and
                          [bytes([b]) for b in universe if re.fullmatch(pat[k:e + 1], bytes([b]))])
            out += b"(" + b"|".join(sorted(members)).replace(b"\n", b"\\n") + b")"
            k = e + 1
        elif c == b".":
            out += b"(a|b|c)"
            k += 1
        else:
            out += c
            k += 1
    return out


@pytest.mark.parametrize("seed", range(20))
def test_char_sets_count_like_unions(seed):
    # a set leaf stands for a union of its bytes: over texts of those bytes the
    # two REs have the same language and the same number of trees (a union of
    # distinct single bytes adds no ambiguity), while the set form has fewer
    # segments
    rng = np.random.default_rng(8000 + seed)
    pat = _tiny_set_re(rng)
    if b"[" not in pat and b"." not in pat:
        pytest.skip("no set leaf")
    o1, o2 = Oracle(pat), Oracle(_expand_sets(pat))
    assert o1.nseg <= o2.nseg
    for x in _strings("abc", 6):
        _, a1, c1, p1 = o1.parse_full(x)
        _, a2, c2, p2 = o2.parse_full(x)
        assert (a1, c1, p1) == (a2, c2, p2), (pat, x)


def test_char_set_segment_text_and_labels():
    o = Oracle(b"([a-e]x|[d-g]y|.z|[^\\x00-\\xfe])*")
    texts = " ".join(o.segments)
    assert "[a-e]4" in texts and "[d-g]7" in texts and ".10" in texts and "[\\xff]12" in texts
    # the end-letter of every segment matches exactly its set's bytes
    for s, t in enumerate(o.segments):
        last = t.split(" ")[-1]
        if last.startswith("[a-e]"):
            assert o.label_sets[s] == frozenset(b"abcde") and o.labels[s] == -2
        if last.startswith(".1"):
            assert o.label_sets[s] == frozenset(range(256)) - {10}
    # a wildcard does not match the newline
    assert o.parse(b"az")[1] and not o.parse(b"\nz")[1]
    with pytest.raises(OracleError):
        Oracle(b"[]")
    with pytest.raises(OracleError):
        Oracle(b"[z-a]")
