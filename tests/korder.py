"""The order of the contracted index k in a plan, as the plan description
states it: colexicographic over the P dims (first fastest), or, when the plan
reports a sub-blocked order `k_sub` = {a, b, bx, by}, the (a, b) plane walked
in bands of by values of dim b, each band cut into blocks of bx values of dim
a (the last band and block shorter when an extent is not a multiple), dim a
fastest inside a block, then dim b, then the blocks, then the bands; the
other P dims outside, in P order.  Written from that statement alone, for the
tests: it shares nothing with the library."""


def p_digits(dims, k_sub):
    """Per linear k, the digit of every P dim (a list of lists)."""
    lens = [d["len"] for d in dims]
    total = 1
    for n in lens:
        total *= n
    if not k_sub:
        out = []
        for lin in range(total):
            dig, r = [], lin
            for n in lens:
                dig.append(r % n)
                r //= n
            out.append(dig)
        return out
    a, b, bx, by = k_sub["a"], k_sub["b"], k_sub["bx"], k_sub["by"]
    La, Lb = lens[a], lens[b]
    others = [i for i in range(len(lens)) if i not in (a, b)]
    plane = []
    for b0 in range(0, Lb, by):
        for a0 in range(0, La, bx):
            for vb in range(b0, min(b0 + by, Lb)):
                for va in range(a0, min(a0 + bx, La)):
                    plane.append((va, vb))
    rest_total = total // (La * Lb) if La * Lb else 0
    out = []
    for rest in range(rest_total):
        rdig, r = {}, rest
        for i in others:
            rdig[i] = r % lens[i]
            r //= lens[i]
        for va, vb in plane:
            dig = [0] * len(lens)
            dig[a], dig[b] = va, vb
            for i in others:
                dig[i] = rdig[i]
            out.append(dig)
    return out


def p_label_values(dims, k_sub, extents):
    """Per linear k, the value of every original label (folded dims cover
    several labels, first fastest)."""
    out = []
    for dig in p_digits(dims, k_sub):
        vals = {}
        for x, v in zip(dims, dig):
            for l in x["labels"]:
                n = extents[l]
                vals[l] = v % n
                v //= n
        out.append(vals)
    return out
