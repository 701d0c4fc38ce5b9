"""Closed-form graphs with known hop distances, used to pin the oracle and to
exercise the GPU path on shapes whose answer is known without any search.

Each builder returns (n, src, dst, dist_fn) where dist_fn(s) gives the exact
distance vector from s by formula (-1 where unreachable).
"""
import numpy as np


def path(n):
    src = np.arange(n - 1, dtype=np.int32)
    dst = src + 1
    return n, src, dst, lambda s: np.abs(np.arange(n) - s).astype(np.int32)


def cycle(n):
    src = np.arange(n, dtype=np.int32)
    dst = ((src + 1) % n).astype(np.int32)

    def dist(s):
        d = np.abs(np.arange(n) - s)
        return np.minimum(d, n - d).astype(np.int32)
    return n, src, dst, dist


def star(k):
    """Hub 0 with leaves 1..k."""
    n = k + 1
    src = np.zeros(k, dtype=np.int32)
    dst = np.arange(1, n, dtype=np.int32)

    def dist(s):
        d = np.full(n, 2 if s != 0 else 1, dtype=np.int32)
        d[0] = 0 if s == 0 else 1
        d[s] = 0
        return d
    return n, src, dst, dist


def complete(n):
    i, j = np.triu_indices(n, 1)

    def dist(s):
        d = np.ones(n, dtype=np.int32)
        d[s] = 0
        return d
    return n, i.astype(np.int32), j.astype(np.int32), dist


def complete_bipartite(a, b):
    n = a + b
    i, j = np.meshgrid(np.arange(a), np.arange(a, n), indexing="ij")

    def dist(s):
        side = np.arange(n) < a
        d = np.where(side == (s < a), 2, 1).astype(np.int32)
        d[s] = 0
        return d
    return n, i.ravel().astype(np.int32), j.ravel().astype(np.int32), dist


def binary_tree(levels):
    """Complete binary tree with 2^levels - 1 vertices; children of i are 2i+1, 2i+2."""
    n = (1 << levels) - 1
    child = np.arange(1, n, dtype=np.int32)
    par = ((child - 1) // 2).astype(np.int32)

    def dist(s):
        assert s == 0
        return np.floor(np.log2(np.arange(n) + 1)).astype(np.int32)
    return n, par, child, dist


def grid(r, c):
    idx = np.arange(r * c).reshape(r, c)
    src = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()]).astype(np.int32)
    dst = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()]).astype(np.int32)

    def dist(s):
        sr, sc = divmod(s, c)
        rr, cc = np.divmod(np.arange(r * c), c)
        return (np.abs(rr - sr) + np.abs(cc - sc)).astype(np.int32)
    return r * c, src, dst, dist


def hypercube(k):
    n = 1 << k
    v = np.arange(n)
    src, dst = [], []
    for b in range(k):
        u = v[(v >> b) & 1 == 0]
        src.append(u)
        dst.append(u | (1 << b))
    src = np.concatenate(src).astype(np.int32)
    dst = np.concatenate(dst).astype(np.int32)

    def dist(s):
        x = np.arange(n) ^ s
        return np.array([bin(int(t)).count("1") for t in x], dtype=np.int32)
    return n, src, dst, dist


def disjoint_paths(n1, n2):
    """Path on [0, n1) and path on [n1, n1+n2): the other component is unreachable."""
    a = np.arange(n1 - 1)
    b = np.arange(n1, n1 + n2 - 1)
    src = np.concatenate([a, b]).astype(np.int32)
    dst = src + 1
    n = n1 + n2

    def dist(s):
        d = np.full(n, -1, dtype=np.int32)
        if s < n1:
            d[:n1] = np.abs(np.arange(n1) - s)
        else:
            d[n1:] = np.abs(np.arange(n1, n) - s)
        return d
    return n, src, dst, dist


def two_cliques_path(k, plen):
    """Cliques on [0,k) and [k,2k); vertex k-1 joined to vertex k by a path of
    plen extra vertices [2k, 2k+plen). Distances from vertex 0."""
    n = 2 * k + plen
    i, j = np.triu_indices(k, 1)
    src = [i, i + k]
    dst = [j, j + k]
    chain = [k - 1] + list(range(2 * k, 2 * k + plen)) + [k]
    src.append(np.array(chain[:-1]))
    dst.append(np.array(chain[1:]))
    src = np.concatenate(src).astype(np.int32)
    dst = np.concatenate(dst).astype(np.int32)

    def dist(s):
        assert s == 0
        d = np.empty(n, dtype=np.int32)
        d[:k] = 1
        d[0] = 0
        d[2 * k:] = 1 + np.arange(1, plen + 1)      # path vertices after k-1
        d[k] = 1 + plen + 1                         # far clique's entry vertex
        d[k + 1:2 * k] = d[k] + 1
        return d
    return n, src, dst, dist


def all_closed_forms():
    """(name, n, src, dst, dist_fn, sources) for every shape."""
    out = []
    for name, (n, s, d, f), srcs in [
        ("path40", path(40), [0, 17, 39]),
        ("cycle33", cycle(33), [0, 5]),
        ("cycle64", cycle(64), [63]),
        ("star50", star(50), [0, 7]),
        ("k12", complete(12), [0, 11]),
        ("k7_9", complete_bipartite(7, 9), [0, 10]),
        ("btree6", binary_tree(6), [0]),
        ("grid9x13", grid(9, 13), [0, 60]),
        ("hypercube7", hypercube(7), [0, 77]),
        ("disjoint", disjoint_paths(10, 15), [3, 20]),
        ("cliques", two_cliques_path(9, 5), [0]),
    ]:
        out.append((name, n, s, d, f, srcs))
    return out
