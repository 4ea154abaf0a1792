"""Parity of the HIP path (through the C ABI) with the serial CPU oracle.

Bit-exact on every column word, the accept flag and the tree count modulo
2^64 and modulo 2^61 - 1, over the paper's worked examples, the plain-small workload, random REs
and texts (accepted and rejected), every lane-chunk size from one window to
the whole text, both table placements, and the edge cases (empty text, one
byte, ragged last chunk, bytes outside the alphabet).
"""
import sys

import numpy as np
import pytest

from gen import regen, textgen
from gpu_util import gpu_parse, to_device
from oracle.oracle import Oracle

S = pytest.importorskip("paper_2503_06763_amd")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check(pat, text, chunk_bytes=0, force_l2=False, o=None, p=None):
    o = o or Oracle(pat)
    p = p or S.Parser(pat)
    say("case", pat[:60] if isinstance(pat, str) else pat[:60], "n=%d" % len(text), "k=%d" % chunk_bytes,
        "l2=%d" % force_l2)
    cols, acc, cnt, cntp = o.parse_full(text)
    g = gpu_parse(p, text, chunk_bytes=chunk_bytes, force_l2=force_l2)
    gcols, gacc, gcnt, gst = g
    assert gcols.shape == cols.shape
    bad = np.nonzero((gcols != cols).any(axis=1))[0]
    assert bad.size == 0, "first differing column %d of %d" % (bad[0], len(text) + 1)
    assert gacc == acc
    assert gst == 0 and gcnt == cnt and g.countp == cntp, (gst, gcnt, cnt, g.countp, cntp)
    return o, p


def test_worked_examples():
    check("(ab|a)*", b"abaaba")
    check("(ab|a)*", b"ab")
    check("(a|b|ab)+", b"abab")
    check("(a|ab|aba)+", b"aba")
    check("(a|())b", b"b")


def test_empty_and_tiny_texts():
    for pat in ["(ab|a)*", "a(b|c)", "(a|b|ab)+"]:
        o, p = Oracle(pat), S.Parser(pat)
        for t in [b"", b"a", b"b", b"ab", b"z"]:
            check(pat, t, o=o, p=p)


def test_plain_small_workload():
    tree = regen.plain_small_re()
    pat = regen.to_re(tree).decode()
    text = textgen.sample_text(tree, 1, 65536).tobytes()
    o, p = Oracle(pat), S.Parser(pat)
    check(pat, text, chunk_bytes=((len(text) + 7) // 8 + 63) // 64 * 64, o=o, p=p)   # 8 chunks
    for k in (64, 128, 1024, 4096, 65536, 1 << 17):
        check(pat, text, chunk_bytes=k, o=o, p=p)
    check(pat, text, chunk_bytes=256, force_l2=True, o=o, p=p)


@pytest.mark.parametrize("seed", range(12))
def test_random_res_and_texts(seed):
    rng = np.random.default_rng(seed)
    alpha = [b"ab", b"abc", b"abcdefghijklmnopqrstuvwxyz"][seed % 3]
    depth = int(rng.integers(4, 8))
    tree = regen.random_re(200 + seed, n_ops=int(rng.integers(6, 4 * depth)), max_depth=depth, alphabet=alpha)
    pat = regen.to_re(tree)
    p = S.Parser(pat)
    o = Oracle(pat)
    n = int(rng.integers(1, 20000))
    text = textgen.sample_text(tree, seed, n).tobytes()
    check(pat, text, chunk_bytes=64 * int(rng.integers(1, 40)), o=o, p=p)
    # corrupted: one byte flipped (usually rejected), and a byte outside the alphabet
    bad = bytearray(text)
    if bad:
        bad[int(rng.integers(len(bad)))] = alpha[int(rng.integers(len(alpha)))]
        check(pat, bytes(bad), chunk_bytes=128, o=o, p=p)
        bad[len(bad) // 2] = 0xff
        check(pat, bytes(bad), chunk_bytes=64, o=o, p=p)


def test_motif_re_counts():
    tree = regen.motif_re()
    pat = regen.to_re(tree)
    text = textgen.sample_text(tree, 3, 30000).tobytes()
    o, p = Oracle(pat), S.Parser(pat)
    for k in (64, 448, 4096):
        check(pat, text, chunk_bytes=k, o=o, p=p)


@pytest.mark.parametrize("flags", [0, S.PARSE_EDGE_SHIFT])
def test_join_trace_matches_oracle_columns(flags):
    """J and J^ at every lane-chunk edge equal the serial forward and backward
    columns there (Eq. joiner reproduces Eq. matrixmul at the chunk edges),
    also when the runs and the join start at shifted edges."""
    tree = regen.plain_small_re()
    pat = regen.to_re(tree).decode()
    text = textgen.sample_text(tree, 7, 5000).tobytes()
    o, p = Oracle(pat), S.Parser(pat)
    k = 192
    gcols, gacc, gcnt, gst, tr = gpu_parse(p, text, chunk_bytes=k, trace=True, flags=flags)
    n = len(text)
    fwd = [o.I]
    for a in text:
        fwd.append(o.step_fwd(fwd[-1], a))
    bwd = [o.F]
    for a in reversed(text):
        bwd.append(o.step_bwd(bwd[-1], a))
    bwd.reverse()
    c = (n + k - 1) // k
    for b in range(c + 1):
        pos = min(b * k, n)
        assert o.to_set(tr[0, b]) == fwd[pos], b
        assert o.to_set(tr[1, b]) == bwd[pos], b


def test_chunking_invariance_all_sizes():
    tree = regen.random_re(11, n_ops=20, max_depth=5, alphabet=b"abc")
    pat = regen.to_re(tree)
    text = textgen.sample_text(tree, 5, 3000).tobytes()
    o, p = Oracle(pat), S.Parser(pat)
    ref = gpu_parse(p, text, chunk_bytes=1 << 16)
    for k in range(64, 3200, 64):
        g = gpu_parse(p, text, chunk_bytes=k)
        assert np.array_equal(g[0], ref[0]) and g[1:] == ref[1:], k
    check(pat, text, chunk_bytes=64, o=o, p=p)


def test_argument_errors():
    import torch
    p = S.Parser("(ab|a)*")
    t = to_device(b"abab" * 10)
    cols = torch.empty((41, p.W), dtype=torch.int64, device=t.device)
    sc = torch.empty(4, dtype=torch.int64, device=t.device)
    with pytest.raises(S.SlpfError) as e:       # capacity
        p.parse_into(t, 40, cols[:10], sc)
    assert e.value.status == S.E_CAPACITY
    with pytest.raises(S.SlpfError) as e:       # chunk size not a multiple of 64
        p.parse_into(t, 40, cols, sc, chunk_bytes=100)
    assert e.value.status == S.E_ARG
    big = torch.empty(64, dtype=torch.uint8, device=t.device)
    with pytest.raises(S.SlpfError) as e:       # misaligned text
        p.parse_into(big[1:], 40, cols, sc)
    assert e.value.status == S.E_ARG


def test_tree_count_paths():
    """Tree counts through every count path: rank-1 chunks (a singleton clean
    column inside), chunks with no singleton column (e.g. (a|b|ab)+ on abab...),
    columns above 16 segments, and the mixtures at chunk edges."""
    cases = [
        ("(a|b|ab)+", b"ab" * 1500, (64, 128, 192, 4096)),           # no singleton column at all
        ("(a|b|ab)+", b"ab" * 31 + b"a", (64,)),                      # 2^31 trees
        ("(a|b|ab)+", (b"ab" * 40 + b"b") * 30, (64, 256)),
        ("(a|ab|b)*(c|bc)+(a|b)*", None, (64, 512, 8192)),
    ]
    tree3 = regen.random_re(3)
    cases.append((regen.to_re(tree3), textgen.sample_text(tree3, 3, 60000).tobytes(), (64, 1024, 4160)))
    motif = regen.motif_re()
    cases.append((regen.to_re(motif), textgen.sample_text(motif, 1, 40000).tobytes(), (64, 320, 4096)))
    for pat, text, ks in cases:
        if text is None:
            text = textgen.sample_text(regen.plain_small_re(), 9, 20000).tobytes()
        o, p = Oracle(pat), S.Parser(pat)
        for k in ks:
            check(pat, text, chunk_bytes=k, o=o, p=p)


def test_recognizer_mode():
    # forward reach and forward join only: the accept flag of every text equals
    # the oracle's, alone and in a batch; no column is written
    import torch
    from gpu_util import device
    device()
    cases = [("(ab|a)*", [b"", b"a", b"abaaba", b"b", b"abb", b"z"]),
             (regen.to_re(regen.plain_small_re()).decode(), None)]
    tree = regen.plain_small_re()
    base = textgen.sample_text(tree, 3, 20000).tobytes()
    cases[1] = (cases[1][0], [base, base[:-1], base[:1000], base[:5000] + b"a" + base[5001:], b"c", b"abc"])
    for seed in (3, 7):
        rt = regen.random_re(400 + seed, n_ops=14, max_depth=5, alphabet=b"abcd")
        x = textgen.sample_text(rt, seed, 9000)
        cases.append((regen.to_re(rt).decode(), [x.tobytes(), textgen.corrupt(x, seed, 0.01, (1, 8)).tobytes()]))
    for pat, texts in cases:
        o, p = Oracle(pat), S.Parser(pat)
        want = [o.parse(t)[1] for t in texts]
        for k in (0, 64, 512):
            got = []
            for t in texts:
                sc = p.recognize(to_device(t), chunk_bytes=k)
                torch.cuda.synchronize()
                s = sc.cpu().numpy().view(np.uint64)
                got.append(bool(s[0]))
                assert int(s[1]) == 0 and int(s[2]) == 2
            assert got == want, (pat[:40], k, got, want)
        # batched recogniser
        dts = [to_device(t) for t in texts]
        sc = torch.zeros((len(texts), 4), dtype=torch.int64, device="cuda:0")
        p.parse_batch_into([(d, len(t), None, sc[j]) for j, (d, t) in enumerate(zip(dts, texts))],
                           flags=S.PARSE_RECOGNIZE)
        torch.cuda.synchronize()
        assert [bool(v) for v in sc[:, 0].cpu().tolist()] == want


def test_next_byte_entries_give_the_same_slpf():
    # speculation from every segment whose end-letter is the chunk's first
    # byte (no previous-byte filter): more runs, the same join results, so
    # the same SLPF, accept flag and count as the reduced entry lists and the
    # oracle; recogniser mode too
    import torch
    from gpu_util import device, gpu_parse
    device()
    cases = []
    for seed in (1, 4, 9):
        rt = regen.random_re(500 + seed, n_ops=14, max_depth=5, alphabet=b"abcd")
        x = textgen.sample_text(rt, seed, 12000)
        cases.append((regen.to_re(rt).decode(), [x.tobytes(), textgen.corrupt(x, seed, 0.01, (1, 8)).tobytes(),
                                                 x.tobytes()[:100], b""]))
    tree = regen.plain_small_re()
    cases.append((regen.to_re(tree).decode(), [textgen.sample_text(tree, 5, 30000).tobytes()]))
    for pat, texts in cases:
        o, p = Oracle(pat), S.Parser(pat)
        assert p.info.max_entries_next_byte >= p.info.max_entries
        for t in texts:
            cols, acc, cnt = o.parse(t)
            for k in (64, 0):
                g = gpu_parse(p, t, chunk_bytes=k, flags=S.PARSE_NEXT_BYTE_ENTRIES)
                assert np.array_equal(g[0], cols), (pat[:40], len(t), k)
                assert g[1] == acc and g[3] == 0 and g[2] == cnt
                sc = torch.zeros(4, dtype=torch.int64, device="cuda:0")
                p.parse_into(to_device(t), len(t), None, sc, k, S.PARSE_RECOGNIZE | S.PARSE_NEXT_BYTE_ENTRIES)
                torch.cuda.synchronize()
                assert bool(sc.cpu().numpy()[0]) == acc


def _max_candidates(o, alpha):
    """Longest candidate (entry) list of the oracle's automaton over byte pairs."""
    best = 0
    for a in [None] + list(alpha):
        for b in list(alpha) + [None]:
            best = max(best, len(o.candidates(a, b)))
    return best


def test_entry_lists_over_64_segments():
    # 4-letter REs whose entry lists hold 65 to 200 segments (chosen on the
    # oracle's own candidate lists): the join masks take several words; texts
    # sampled from the language, corrupted ones, lane chunks from one window up
    found = []
    seed = 900
    while len(found) < 4 and seed < 1400:
        seed += 1
        try:
            tree = regen.random_re(seed, n_ops=int(14 + seed % 17), max_depth=6, alphabet=b"ACGT")
        except RuntimeError:
            continue
        pat = regen.to_re(tree)
        o = Oracle(pat)
        e = _max_candidates(o, b"ACGT")
        if 64 < e <= 200:
            found.append((tree, pat, o, e))
    assert len(found) == 4
    for tree, pat, o, e in found:
        p = S.Parser(pat)
        assert p.info.max_entries == e
        say("wide entry lists", e, pat[:60])
        text = textgen.sample_text(tree, 3, 12000).tobytes()
        for k in (64, 256, 0):
            check(pat, text, chunk_bytes=k, o=o, p=p)
        bad = textgen.corrupt(np.frombuffer(text, np.uint8), 5, 0.01, (1, 8)).tobytes()
        check(pat, bad, chunk_bytes=128, o=o, p=p)
        # the compact SLPF has no one-word form for such lists
        with pytest.raises(S.SlpfError) as err:
            p.parse_compact(to_device(text))
        assert err.value.status == S.E_TOO_LARGE


@pytest.mark.parametrize("seed", range(10))
def test_char_set_res_and_texts(seed):
    # leaves that are character sets or the wildcard (App. A, character
    # features); alphabets of 4, 10 and 128 byte values; accepted and
    # corrupted texts; several lane-chunk sizes and both table placements
    rng = np.random.default_rng(600 + seed)
    alpha = [b"abcd", b"abcdefghij", bytes(range(1, 128))][seed % 3]
    depth = int(rng.integers(4, 7))
    s = 6100 + seed
    while True:
        try:
            tree = regen.random_re(s, n_ops=int(rng.integers(6, 4 * depth)), max_depth=depth,
                                   alphabet=alpha, set_p=0.5, max_tries=200)
            break
        except RuntimeError:
            s += 100
    pat = regen.to_re(tree)
    o, p = Oracle(pat), S.Parser(pat)
    assert p.segments == o.segments
    n = int(rng.integers(1, 30000))
    text = textgen.sample_text(tree, seed, n)
    check(pat, text.tobytes(), chunk_bytes=64 * int(rng.integers(1, 40)), o=o, p=p)
    bad = textgen.corrupt(text, seed, frac=0.01, block=(1, 16)).tobytes()
    check(pat, bad, chunk_bytes=64, o=o, p=p)
    check(pat, text.tobytes(), chunk_bytes=128, force_l2=True, o=o, p=p)
    check(pat, b"", o=o, p=p)


def _as_unions(node):
    """The same tree with every character set written as a union of its bytes."""
    k = node[0]
    if k == 'set':
        return regen.lit_union(node[1])
    if k in ('cat', 'alt'):
        return (k, [_as_unions(c) for c in node[1]])
    if k in ('star', 'plus', 'opt'):
        return (k, _as_unions(node[1]))
    return node


@pytest.mark.parametrize("seed", range(4))
def test_char_set_and_union_forms_count_alike(seed):
    # a character set is one terminal for any one of its bytes: an RE and the
    # same RE with its sets written as unions of single bytes have the same
    # language and the same number of trees (each byte matches exactly one
    # branch of the union), the set form with fewer segments.  Random
    # ambiguous REs and, for seed 0, the CSV record RE; each form bit-exact
    # against its own oracle
    if seed == 0:
        tree = regen.csv_record_re(sets=True)
        text = textgen.csv_record_text(17, 200000)
    else:
        s = 6500 + seed
        while True:
            tree = regen.random_re(s, n_ops=12, max_depth=5, alphabet=b"abcd", set_p=0.6)
            if regen.WILDCARD not in [x[1] for x in _leaves(tree)]:
                break
            s += 100
        text = textgen.sample_text(tree, seed, 20000)
    us, ss = regen.to_re(_as_unions(tree)), regen.to_re(tree)
    pu, ps = S.Parser(us), S.Parser(ss)
    assert ps.info.num_segments < pu.info.num_segments
    ou, os_ = Oracle(us), Oracle(ss)
    bad = textgen.corrupt(text, 18, frac=0.01, block=(4, 64))
    for t in (text.tobytes(), bad.tobytes()):
        check(us, t, o=ou, p=pu)
        check(ss, t, o=os_, p=ps)
        a, b = gpu_parse(pu, t), gpu_parse(ps, t)
        assert (a[1], a[2], a.countp) == (b[1], b[2], b.countp)


def _leaves(node):
    if node[0] in ('lit', 'set', 'eps'):
        return [node]
    if node[0] in ('cat', 'alt'):
        return [x for c in node[1] for x in _leaves(c)]
    return _leaves(node[1])


@pytest.mark.parametrize("seed", range(8))
def test_chunk_edge_shifting(seed):
    # chunk-edge shifting (Sect. Tool optimization, technique (ii)) forced on
    # and off: the same columns, accept flag and counts as the oracle, over
    # random REs (with and without character sets), accepted and corrupted
    # texts, several lane-chunk sizes (so shift windows of 32 to 256 bytes)
    # and both table placements
    rng = np.random.default_rng(900 + seed)
    alpha = [b"abc", b"abcdefghij", b"abcdefghijklmnopqrstuvwxyz"][seed % 3]
    s = 8100 + seed
    while True:
        try:
            tree = regen.random_re(s, n_ops=int(rng.integers(8, 24)), max_depth=6, alphabet=alpha,
                                   set_p=0.3 if seed % 2 else 0.0, max_tries=200)
            break
        except RuntimeError:
            s += 100
    pat = regen.to_re(tree)
    o, p = Oracle(pat), S.Parser(pat)
    text = textgen.sample_text(tree, seed, int(rng.integers(2000, 40000)))
    bad = textgen.corrupt(text, seed, frac=0.02, block=(1, 32))
    for t in (text.tobytes(), bad.tobytes()):
        cols, acc, cnt, cntp = o.parse_full(t)
        for k in (64, 256, 1024):
            for flags in (S.PARSE_EDGE_SHIFT, S.PARSE_NO_EDGE_SHIFT):
                for l2 in ((False, True) if k == 256 else (False,)):
                    say("shift", pat[:50], "n=%d k=%d flags=%d l2=%d" % (len(t), k, flags, l2))
                    g = gpu_parse(p, t, chunk_bytes=k, flags=flags, force_l2=l2)
                    bad_cols = np.nonzero((g[0] != cols).any(axis=1))[0]
                    assert bad_cols.size == 0, "first differing column %d" % bad_cols[0]
                    assert g[1] == acc and g[3] == 0 and g[2] == cnt and g.countp == cntp


def test_chunk_edge_shifting_record_text():
    # record text: every shifted edge lands just after a newline, where the
    # entry list has a single segment; batched texts and the recogniser too
    pat = regen.to_re(regen.record_re())
    o, p = Oracle(pat), S.Parser(pat)
    text = textgen.record_text(77, 300000)
    for t in (text.tobytes(), textgen.corrupt(text, 78, frac=0.01, block=(4, 64)).tobytes()):
        cols, acc, cnt, cntp = o.parse_full(t)
        for k in (256, 4096):
            for flags in (0, S.PARSE_NO_EDGE_SHIFT):
                g = gpu_parse(p, t, chunk_bytes=k, flags=flags)
                bad_cols = np.nonzero((g[0] != cols).any(axis=1))[0]
                assert bad_cols.size == 0, "k=%d flags=%d: first differing column %d" % (k, flags, bad_cols[0])
                assert g[1] == acc and g[3] == 0 and g[2] == cnt and g.countp == cntp
        r = p.recognize(to_device(t), chunk_bytes=256)
        assert bool(int(r[0].item())) == acc


@pytest.mark.parametrize("seed", range(6))
def test_all_dfa_states_speculation(seed):
    # the standard speculation the paper compares ME-DFA entries with (Sect.
    # 5): runs from every DFA state at the inner lane-chunk edges.  Same
    # columns, accept flag and counts as the oracle; several chunk sizes
    rng = np.random.default_rng(950 + seed)
    alpha = [b"ab", b"abc", b"abcdefghijklmnopqrstuvwxyz"][seed % 3]
    tree = regen.random_re(8600 + seed, n_ops=int(rng.integers(8, 20)), max_depth=6, alphabet=alpha)
    pat = regen.to_re(tree)
    o, p = Oracle(pat), S.Parser(pat)
    text = textgen.sample_text(tree, seed, int(rng.integers(3000, 30000)))
    bad = textgen.corrupt(text, seed, frac=0.02, block=(1, 32))
    for t in (text.tobytes(), bad.tobytes(), text.tobytes()[:70]):
        cols, acc, cnt, cntp = o.parse_full(t)
        for k in (64, 512):
            say("alldfa", pat[:50], "n=%d k=%d" % (len(t), k))
            g = gpu_parse(p, t, chunk_bytes=k, flags=S.PARSE_ALL_DFA_STATES)
            bad_cols = np.nonzero((g[0] != cols).any(axis=1))[0]
            assert bad_cols.size == 0, "first differing column %d" % bad_cols[0]
            assert g[1] == acc and g[3] == 0 and g[2] == cnt and g.countp == cntp


def test_all_dfa_states_trace_and_recognizer():
    # J and J^ at every edge, and the recogniser, with the all-DFA-states lists
    tree = regen.plain_small_re()
    pat = regen.to_re(tree).decode()
    text = textgen.sample_text(tree, 7, 5000).tobytes()
    o, p = Oracle(pat), S.Parser(pat)
    k = 192
    g = gpu_parse(p, text, chunk_bytes=k, trace=True, flags=S.PARSE_ALL_DFA_STATES)
    tr = g[4]
    fwd = [o.I]
    for a in text:
        fwd.append(o.step_fwd(fwd[-1], a))
    bwd = [o.F]
    for a in reversed(text):
        bwd.append(o.step_bwd(bwd[-1], a))
    bwd.reverse()
    n = len(text)
    for b in range((n + k - 1) // k + 1):
        pos = min(b * k, n)
        assert o.to_set(tr[0, b]) == fwd[pos], b
        assert o.to_set(tr[1, b]) == bwd[pos], b
    import torch
    sc = torch.empty(4, dtype=torch.int64, device="cuda:0")
    for t in (text, text[:-1] + b"z"):
        p.parse_into(to_device(t), len(t), None, sc, 256, S.PARSE_RECOGNIZE | S.PARSE_ALL_DFA_STATES)
        assert bool(int(sc[0].item())) == o.parse_full(t)[1]
