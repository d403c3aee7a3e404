"""Scheduling of a sampling round on one GPU (oracle side; test infrastructure).

The paper's scheduler (Sec. 3-4) gives tasks to partitions of q_l processors:
  * Alg. incremental_greedy: tasks are taken by decreasing q (the finest level
    first) and each goes to the least-loaded processors;
  * eq. batch: a level's samples are handed out in batches of consecutive
    indices whose size falls with the number still unassigned, between a
    minimum and a maximum fraction of the samples per partition
    ceil(N_l / (p|q_l)).
On one GPU a partition becomes a lane: a stream that solves one batched task
at a time.  The readings (the equation as printed is garbled: its value is
always 1) are
  * partitions of every level: the K lanes, so p|q_l = K;
  * b = ceil((N - n) / K), kept between ceil(0.01 ceil(N / K)) and
    ceil(phi^-1 ceil(N / K)) (phi the golden ratio), the defaults the paper
    states, where N is the number of samples the round assigns to the level
    and n those already assigned; the minimum is raised to min(cap, fill),
    cap being the lane capacity of the level and fill the samples that fill
    the device (a property of the GPU's kernels, given as an input here);
    every batch is capped by cap and by what is left;
  * with one lane there is no other partition to leave work for: batches are
    the capacity;
  * a batch of a level l > 0 is two solves, on the level's mesh and on the
    coarse mesh of its pair (Sec. 2.2); optionally the solves of two levels on
    one mesh share a task (see plan); a task's work is its samples times the
    interior unknowns of its mesh;
  * tasks are ordered by decreasing mesh (q of the task), then by decreasing
    level, then in sample order; each goes to the lane with the least work
    assigned so far, the lowest lane on ties.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

PHI_INV = (math.sqrt(5.0) - 1.0) / 2.0


def dofs(n: int) -> int:
    return (n - 1) ** 3


def batch_sizes(count: int, lanes: int, cap: int, fill: int) -> List[int]:
    """Batch sizes of one level's share of a round (eq. batch as read above)."""
    if lanes <= 1:
        out, left = [], count
        while left > 0:
            out.append(min(left, cap))
            left -= out[-1]
        return out
    per = -(-count // lanes)
    most = math.ceil(per * PHI_INV)
    least = max(-(-per // 100), min(cap, max(1, fill)))
    out, left = [], count
    while left > 0:
        b = -(-left // lanes)
        b = max(least, min(most, b))
        b = min(b, cap, left)
        out.append(b)
        left -= b
    return out


def level_cap(n0: int, levels: int, level: int, max_batch: int, limit: int = 65536) -> int:
    """Samples a lane takes of a level: max_batch on the finest mesh and as many
    as cost the same interior unknowns (pair of meshes) on a coarser level, at
    most `limit`, never below max_batch."""
    def pair(l):
        n = n0 << l
        return dofs(n) + (dofs(n // 2) if l > 0 else 0)
    cap = min(max_batch * max(1.0, pair(levels - 1) / pair(level)), float(limit))
    return max(max_batch, int(cap))


def plan(n0: int, requests: Sequence[Tuple[int, int, int]], lanes: int, caps: Sequence[int],
         fills: Sequence[int], pack: bool = False):
    """Tasks of a round: requests are (level, first, count); caps[m] and
    fills[m] the lane capacity and the device-filling batch of level m (whose
    own mesh is n0 << m), indexed by level.  With `pack`, the coarse solves of
    level m+1 and the fine solves of level m (both on mesh n0 << m) are paired
    in order, the i-th with the i-th, into one task when together they fit
    caps[m]; without it a mesh's coarse solves come before its fine ones.
    Returns the tasks in assignment order, each a dict (n, lane, parts), parts
    being dicts (level, first, count) in their order within the task."""
    levels = len(caps)
    coarse = [[] for _ in range(levels)]
    fine = [[] for _ in range(levels)]
    for level, first, count in sorted(requests, key=lambda q: -q[0]):
        off = 0
        for b in batch_sizes(count, lanes, caps[level], fills[level]):
            part = dict(level=level, first=first + off, count=b)
            fine[level].append(part)
            if level > 0:
                coarse[level - 1].append(dict(part))
            off += b
    tasks = []
    for m in range(levels - 1, -1, -1):
        a, f = coarse[m], fine[m]
        if not pack:
            groups = [[p] for p in a] + [[p] for p in f]
        else:
            groups = []
            for i in range(max(len(a), len(f))):
                if i < len(a) and i < len(f) and a[i]["count"] + f[i]["count"] <= caps[m]:
                    groups.append([a[i], f[i]])
                else:
                    groups += [[a[i]]] if i < len(a) else []
                    groups += [[f[i]]] if i < len(f) else []
        for g in groups:
            tasks.append(dict(n=n0 << m, parts=g, count=sum(p["count"] for p in g)))
    load = [0] * max(1, lanes)
    for t in tasks:
        lane = min(range(len(load)), key=lambda i: (load[i], i))
        t["lane"] = lane
        load[lane] += t["count"] * dofs(t["n"])
    return tasks


def flat(tasks):
    """(level, n, first, count, lane, task) of every part, tasks in order."""
    return [(p["level"], t["n"], p["first"], p["count"], t["lane"], i)
            for i, t in enumerate(tasks) for p in t["parts"]]
