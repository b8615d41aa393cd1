"""Training data for the learned coarse-space preconditioner.

A *system* is the damped reduced system of one BA problem at one lambda, as
the library produces it: the block graph with its node and edge inputs
(ba_export_gnn_graph), the gauge rows of each node (ba_export_gauge_basis)
and the blocks of S on the graph's nodes and edges (from
ba_export_schur_dense).  `make_batch` packs several systems into the
ba_gnn_batch layout: nodes sorted by type over the whole batch, edges
sorted by destination, each edge's reverse indexed.  This is host-side data
layout only; every number comes from the library.
"""
from __future__ import annotations

import numpy as np

from .binding import GNNBatch


def system_from_handle(ba, lam):
    """Linearise at lam and read the system (dict of numpy arrays)."""
    ba.linearize(lam)
    g = ba.export_gnn_graph()
    S = ba.export_schur_dense()
    S = 0.5 * (S + S.T)
    return system_from_dense(g, S, ba.export_gauge_basis())


def system_from_dense(g, S, gauge):
    """Attach the node and edge blocks of a dense S and the gauge rows
    (n_A x 7) of each node to graph arrays g."""
    n = len(g["node_type"])
    off = np.asarray(g["node_off"], dtype=np.int64)
    size = np.array([int(np.count_nonzero(g["node_unit"][i])) for i in range(n)], dtype=np.int64)
    s_node, s_node_off, o = [], np.zeros(n, np.int64), 0
    for i in range(n):
        b = S[off[i]:off[i] + size[i], off[i]:off[i] + size[i]]
        s_node.append(b.ravel())
        s_node_off[i] = o
        o += b.size
    m = len(g["edge_src"])
    s_edge, s_edge_off, o = [], np.zeros(m, np.int64), 0
    for e in range(m):
        i, j = g["edge_dst"][e], g["edge_src"][e]
        b = S[off[i]:off[i] + size[i], off[j]:off[j] + size[j]]
        s_edge.append(b.ravel())
        s_edge_off[e] = o
        o += b.size
    node_gauge = np.zeros((n, 9, gauge.shape[1]))
    for i in range(n):
        node_gauge[i, :size[i]] = gauge[off[i]:off[i] + size[i]]
    out = dict(g)
    out.update(size=size, node_gauge=node_gauge, s_node=np.concatenate(s_node) if s_node else np.zeros(0),
               s_node_off=s_node_off, s_edge=np.concatenate(s_edge) if s_edge else np.zeros(0),
               s_edge_off=s_edge_off, nA=int(S.shape[0]))
    return out


def make_batch(systems, with_s=True) -> GNNBatch:
    """Pack systems into one batch (nodes of all systems sorted by type)."""
    types = np.concatenate([s["node_type"] for s in systems])
    sys_id = np.concatenate([np.full(len(s["node_type"]), k, np.int32) for k, s in enumerate(systems)])
    local = np.concatenate([np.arange(len(s["node_type"])) for s in systems])
    order = np.lexsort((local, sys_id, types))  # by type, then system, then node
    N = len(order)
    base = np.cumsum([0] + [len(s["node_type"]) for s in systems])
    new_index = np.empty(N, np.int64)
    new_index[order] = np.arange(N)
    node_x = np.concatenate([s["node_x"] for s in systems])[order]
    node_unit = np.concatenate([s["node_unit"] for s in systems])[order]
    src = np.concatenate([new_index[base[k] + s["edge_src"]] for k, s in enumerate(systems)])
    dst = np.concatenate([new_index[base[k] + s["edge_dst"]] for k, s in enumerate(systems)])
    ex = np.concatenate([s["edge_x"] for s in systems]) if len(src) else np.zeros((0, 8), np.float32)
    eorder = np.lexsort((src, dst))
    src, dst, ex = src[eorder], dst[eorder], ex[eorder]
    key = dst * N + src
    rev = np.searchsorted(key, src * N + dst)
    kw = {}
    if with_s:
        s_node = np.concatenate([s["s_node"] for s in systems])
        node_base = np.cumsum([0] + [len(s["s_node"]) for s in systems])
        s_node_off = np.concatenate([s["s_node_off"] + node_base[k] for k, s in enumerate(systems)])[order]
        s_edge = np.concatenate([s["s_edge"] for s in systems])
        edge_base = np.cumsum([0] + [len(s["s_edge"]) for s in systems])
        s_edge_off = np.concatenate([s["s_edge_off"] + edge_base[k] for k, s in enumerate(systems)])[eorder]
        kw = dict(s_node=s_node, s_node_off=s_node_off, s_edge=s_edge if len(s_edge) else np.zeros(1),
                  s_edge_off=s_edge_off, node_gauge=np.concatenate([s["node_gauge"] for s in systems])[order])
    batch = GNNBatch(node_x, types[order], sys_id[order], node_unit, src, dst, rev, ex, len(systems), **kw)
    batch.order = order  # batch node k is input node order[k] (systems concatenated)
    return batch
