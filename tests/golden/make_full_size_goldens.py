"""Write the full-size expected values (accept flag, tree count modulo 2^64
and modulo 2^61 - 1) of the large workloads, computed by the oracle's
DFA-lookup serial parser over each whole text.

The texts are the seeded synthetic workloads the GPU tests parse at full
size (generated here by ``gen/``, never read from the GPU path); the hashes
of the RE and the text are stored so a test can tell that it parses the same
input.  Usage, from the repository root:

    python tests/golden/make_full_size_goldens.py [--only NAME ...]

Takes minutes (the 1 GiB record text the longest); rewrites
tests/golden/full_size_counts.yaml, keeping the entries not recomputed.
"""
import argparse
import hashlib
import os
import sys
import time

import yaml

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
OUT = os.path.join(HERE, "full_size_counts.yaml")


def workloads():
    """name -> (RE bytes, function giving the uint8 text)."""
    from gen import regen, textgen
    tree = regen.random_re(23)
    pat = regen.to_re(tree)

    def clean():
        return textgen.sample_text(tree, 23, 1 << 28)

    def corrupted():
        return textgen.corrupt(clean(), 24, frac=0.05, block=(64, 4096))

    rec = regen.to_re(regen.record_re())
    return {
        "single_re_clean": (pat, clean),
        "single_re_corrupted": (pat, corrupted),
        "record_re": (rec, lambda: textgen.record_text(31, 1 << 30)),
    }


def sha(b) -> str:
    return hashlib.sha256(b).hexdigest()


def main():
    from oracle.oracle import Oracle
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", nargs="*")
    args = ap.parse_args()
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = yaml.safe_load(f) or {}
    for name, (pat, make) in workloads().items():
        if args.only and name not in args.only:
            continue
        text = make()
        t0 = time.time()
        o = Oracle(pat)
        _, acc, cnt, cntp = o.parse_dfa_full(text, [], 0, count=True)
        data[name] = {"re_sha256": sha(pat), "text_bytes": int(text.size), "text_sha256": sha(text.tobytes()),
                      "accepted": bool(acc), "trees_mod_2_64": int(cnt), "trees_mod_2_61_1": int(cntp)}
        print(name, data[name], "%.0f s" % (time.time() - t0), flush=True)
        with open(OUT, "w") as f:
            f.write("# Accept flag and tree counts of the full-size workloads, from the oracle's\n"
                    "# DFA-lookup serial parser over each whole text (make_full_size_goldens.py).\n")
            yaml.safe_dump(data, f, sort_keys=True)


if __name__ == "__main__":
    main()
