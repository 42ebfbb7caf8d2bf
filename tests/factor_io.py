"""Convert an oracle factorization into the import arrays of mbf_import.

Test glue: reads the oracle's factor dictionaries and lays them out in the
order documented in include/mbf.h (mbf_import_desc).  Neither the oracle
nor the library depends on this module.
"""

import numpy as np


def _cm(a):
    return np.asarray(a, np.complex128).ravel(order="F")


def to_import(bf):
    xt, ot, L, m = bf.xt, bf.ot, bf.L, bf.m
    ranks, v, h, s, g, u = [], [], [], [], [], []
    for st in range(L + 1):
        for a in xt.nodes[st]:
            for b in ot.nodes[L - st]:
                ranks.append(bf.rank[st][(int(a), int(b))])
    for b in ot.nodes[L]:
        v.append(_cm(bf.V0[int(b)]))
    for st in range(m):
        for a in xt.nodes[st]:
            for bp in ot.nodes[L - st - 1]:
                for bk in ot.children(L - st - 1, int(bp)):
                    h.append(_cm(bf.H[st][(bk, int(a))]))
    for a in xt.nodes[m]:
        for b in ot.nodes[L - m]:
            s.append(np.asarray(bf.S[(int(a), int(b))], np.float64))
    for st in range(m, L):
        for a in xt.nodes[st]:
            for bp in ot.nodes[L - st - 1]:
                for ac in xt.children(st, int(a)):
                    g.append(_cm(bf.G[st][(ac, int(bp))]))
    for a in xt.nodes[L]:
        u.append(_cm(bf.UL[int(a)]))

    def cat(lst, dt):
        return np.concatenate(lst).astype(dt) if lst else np.zeros(0, dt)

    return dict(depth=L, x_leaf_code=xt.leaf_code, xi_leaf_code=ot.leaf_code,
                ranks=np.asarray(ranks, np.int32), v_leaf=cat(v, np.complex128),
                h_blocks=cat(h, np.complex128), s_mid=cat(s, np.float64),
                g_blocks=cat(g, np.complex128), u_leaf=cat(u, np.complex128))
