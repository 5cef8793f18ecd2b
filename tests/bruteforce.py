"""Brute-force connectivity by breadth-first search (pure Python, tiny graphs).

An independent check of the union-find oracle: components are found by BFS
over an adjacency list of all edges seen so far, starting from vertices in
ascending order, so each component's label is its smallest vertex id.
"""
from collections import deque

import numpy as np


def bfs_labels(n, edges):
    adj = [[] for _ in range(n)]
    for a, b in edges:
        a, b = int(a), int(b)
        if 0 <= a < n and 0 <= b < n:
            adj[a].append(b)
            adj[b].append(a)
    label = [-1] * n
    for s in range(n):
        if label[s] >= 0:
            continue
        label[s] = s
        dq = deque([s])
        while dq:
            x = dq.popleft()
            for y in adj[x]:
                if label[y] < 0:
                    label[y] = s
                    dq.append(y)
    return np.asarray(label, np.int32)


def bfs_answers(labels, pairs):
    n = len(labels)
    out = np.zeros(len(pairs), np.uint8)
    for i, (a, b) in enumerate(pairs):
        a, b = int(a), int(b)
        if 0 <= a < n and 0 <= b < n:
            out[i] = 1 if labels[a] == labels[b] else 0
    return out
