"""Write the frozen hash-spec vectors (tests/golden/hash_spec_vectors.json).

A hand calculator for the library's 64-bit hash spec, in plain Python
integers, written from the spec's definition (HASH_SPEC.md) and the
published SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014; its
published output vector for seed 1234567 is checked here before anything is
written).  It shares nothing with the C oracle or the GPU library: the oracle
is held to these numbers by tests/test_oracle.py, the GPU path by
tests/test_gpu_parity.py.

    python tests/golden/make_hash_vectors.py            # writes the JSON
    python tests/golden/make_hash_vectors.py --markdown # the table of HASH_SPEC.md

The worked graph (vertex: types; out-edges (label, target)):
    v0: {3}        (0, v1), (5, v2), (0, v1)   -- the repeated edge counts once
    v1: {0}        none
    v2: {}         none
    v3: {0, 1}     (5, v2)
    v4: {1, 0, 1}  none                        -- the same type set as v3
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
MASK = (1 << 64) - 1


def M(z: int) -> int:
    """SplitMix64 output function."""
    z &= MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    return z ^ (z >> 31)


def check_published_vector():
    state, inc = 1234567, 0x9E3779B97F4A7C15
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
            16408922859458223821]
    got = []
    for _ in want:
        state = (state + inc) & MASK
        got.append(M(state))
    if got != want:
        raise SystemExit("the mixer does not reproduce the published SplitMix64 vector")


C_T, C_L, C_S, C_E = M(1), M(2), M(3), M(4)


def t_of(types) -> int:
    return M(C_T + sum(M(C_T ^ tau) for tau in sorted(set(types))))


def salt(label: int) -> int:
    return M(C_L + label)


def h_next(t_v: int, pairs) -> dict:
    """One step with every intermediate: pairs = [(label, h_prev(w))]."""
    keys = [hw ^ salt(l) for l, hw in pairs]
    distinct = sorted(set(keys))
    mixed = [M(q ^ C_E) for q in distinct]
    s = sum(mixed) & MASK
    inner = M(C_S + s)
    return {"keys": keys, "distinct_keys": distinct, "mixed": mixed, "sum": s, "inner": inner,
            "h": M(t_v ^ inner)}


TYPES = [[3], [0], [], [0, 1], [1, 0, 1]]
EDGES = [(0, 0, 1), (0, 5, 2), (0, 0, 1), (3, 5, 2)]  # (v, label, w)


def vectors() -> dict:
    v = {"C_T": C_T, "C_L": C_L, "C_S": C_S, "C_E": C_E,
         "M(C_T^0)": M(C_T ^ 0), "M(C_T^1)": M(C_T ^ 1), "M(C_T^3)": M(C_T ^ 3),
         "t({})": t_of([]), "t({0})": t_of([0]), "t({0,1})": t_of([0, 1]), "t({3})": t_of([3]),
         "salt(0)": salt(0), "salt(5)": salt(5)}
    n = len(TYPES)
    t = [t_of(ts) for ts in TYPES]
    levels = [t]
    steps = {}
    for k in (1, 2):
        prev = levels[-1]
        cur = []
        for u in range(n):
            pairs = [(l, prev[w]) for (s, l, w) in EDGES if s == u]
            st = h_next(t[u], pairs)
            steps["h%d(v%d)" % (k, u)] = st
            cur.append(st["h"])
        levels.append(cur)
    v["graph"] = {"types": TYPES, "edges": EDGES}
    v["t"] = t
    v["h1"] = levels[1]
    v["h2"] = levels[2]
    v["steps"] = steps
    return v


def as_json(v: dict) -> dict:
    """Integers as 0x-prefixed 16-digit hex strings (JSON has no u64)."""
    def conv(x):
        if isinstance(x, bool):
            return x
        if isinstance(x, int):
            return "0x%016x" % x
        if isinstance(x, list):
            return [conv(y) for y in x]
        if isinstance(x, dict):
            return {k: conv(y) for k, y in x.items()}
        return x
    out = {k: conv(x) for k, x in v.items() if k != "graph"}
    out["graph"] = v["graph"]
    return out


def markdown(v: dict) -> str:
    rows = ["| quantity | value |", "|---|---|"]
    for k in ("C_T", "C_L", "C_S", "C_E", "M(C_T^0)", "M(C_T^1)", "M(C_T^3)", "t({})", "t({0})", "t({0,1})",
              "t({3})", "salt(0)", "salt(5)"):
        rows.append("| `%s` | `0x%016x` |" % (k, v[k]))
    st = v["steps"]["h1(v0)"]
    for i, q in enumerate(st["keys"]):
        rows.append("| `h1(v0)` key %d | `0x%016x` |" % (i, q))
    for i, f in enumerate(st["mixed"]):
        rows.append("| `h1(v0)` mixed distinct key %d | `0x%016x` |" % (i, f))
    rows.append("| `h1(v0)` sum | `0x%016x` |" % st["sum"])
    rows.append("| `h1(v0)` M(C_S + sum) | `0x%016x` |" % st["inner"])
    for k in (1, 2):
        for u in range(len(TYPES)):
            rows.append("| `h%d(v%d)` | `0x%016x` |" % (k, u, v["h%d" % k][u]))
    return "\n".join(rows)


def main():
    check_published_vector()
    v = vectors()
    if "--markdown" in sys.argv:
        print(markdown(v))
        return
    path = os.path.join(HERE, "hash_spec_vectors.json")
    with open(path, "w") as f:
        json.dump(as_json(v), f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
