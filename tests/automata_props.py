"""Properties of an RE read off the oracle's own automata (test helpers)."""


def column_unambiguous(o):
    """True iff every forward state set reachable from I meets every reverse
    state set reachable from F in at most one segment.  A clean column of an
    accepted text is such an intersection, so then every clean column is a
    single segment and every accepted text has exactly one tree."""
    alpha = sorted(frozenset().union(*o.label_sets))

    def closure(start, step):
        seen, todo = {start}, [start]
        while todo:
            s = todo.pop()
            for a in alpha:
                t = step(s, a)
                if t and t not in seen:
                    seen.add(t)
                    todo.append(t)
        return seen
    fs, bs = closure(o.I, o.step_fwd), closure(o.F, o.step_bwd)
    return max(len(f & b) for f in fs for b in bs) <= 1
