"""Pause-model scheduler stress: the oracle side (test infrastructure only).

Sec. 5.1 ("A benchmarking example") benchmarks the scheduler with a model
whose evaluation only waits for a random time, uniform with mean mu and
spread sqrt(3) sigma on each side (sigma read as a standard deviation: the
section later gives sigma as multiples of mu), and measures the scheduler
through the active ratio A(p) = a(p) / (p t_w(p)) of eq. active_ratio.

This module computes, for the device run of mlmc_pause_model:
  * the durations: sample i of level l waits a + w u microseconds,
    a = mu - sqrt(3) sigma, w = 2 sqrt(3) sigma, u the uniform of word 0 of the
    Philox4x64-10 block with key (seed, 0) and counter (i, l, 0, 1), counted
    in clock ticks as floor(d f + 1/2) for a clock of f MHz;
  * the schedule of those ticks: tasks of `batch` consecutive samples of a
    level, queued finest level first (the finest-first rule of the paper's
    incremental greedy algorithm), admitted at step boundaries in queue order
    whenever their width fits the free slots; a step lasts
    max(min_step, least remaining time of a running task), each running task
    uses min(remaining, step), tasks with nothing left finish at the step's
    end.  `schedule` follows these rules step by step; `event_schedule` is an
    independent event-driven formulation of the same rules used to check it.
Plain Python integers throughout the schedule.
"""
from __future__ import annotations

import heapq
import math

import numpy as np

from . import rng


def law(mu_us: float, sigma_us: float):
    """(a, w): the duration d = a + w u of a sample, u uniform in (0, 1)."""
    s3 = math.sqrt(3.0) * sigma_us
    return mu_us - s3, 2.0 * s3


def durations_us(seed: int, level: int, count: int, mu_us: float, sigma_us: float) -> np.ndarray:
    """Durations (microseconds) of samples 0..count-1 of `level`."""
    a, w = law(mu_us, sigma_us)
    out = np.empty(count, dtype=np.float64)
    for i in range(count):
        word = rng.philox4x64((i, level, 0, 1), (seed, 0))[0]
        u = float(rng.uniforms(np.array([word], dtype=np.uint64))[0])
        out[i] = a + w * u
    return out


def to_ticks(d_us: np.ndarray, clock_mhz: float) -> np.ndarray:
    """Clock ticks of each duration: floor(d f + 1/2)."""
    return np.array([math.floor(float(d) * clock_mhz + 0.5) for d in d_us], dtype=np.int64)


def tasks_of(counts, widths, ticks, batch):
    """Tasks (level, width, first sample, samples, ticks) in queue order: finest level first."""
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    out = []
    for lv in range(len(counts) - 1, -1, -1):
        for i in range(0, int(counts[lv]), batch):
            n = min(batch, int(counts[lv]) - i)
            first = int(off[lv]) + i
            out.append((lv, int(widths[lv]), first, n, int(sum(int(t) for t in ticks[first:first + n]))))
    return out


def schedule(counts, widths, ticks, capacity: int, batch: int, min_step_ticks: int = 0):
    """Step-by-step schedule; returns dict(steps, step_lengths, done_step per sample, active, ideal_ratio)."""
    tasks = tasks_of(counts, widths, ticks, batch)
    rem = [t[4] for t in tasks]
    queue = list(range(len(tasks)))          # queue order
    free = capacity
    running = []
    done = np.full(int(sum(counts)), -1, dtype=np.int64)
    lengths = []
    while True:
        waiting = []
        for q in queue:                        # every queued task that fits, in queue order
            if tasks[q][1] <= free:
                running.append(q)
                free -= tasks[q][1]
            else:
                waiting.append(q)
        queue = waiting
        if not running:
            break
        step = max(min(rem[r] for r in running), min_step_ticks)
        still = []
        for r in running:
            rem[r] -= min(rem[r], step)
            if rem[r] == 0:
                free += tasks[r][1]
                done[tasks[r][2]:tasks[r][2] + tasks[r][3]] = len(lengths)
            else:
                still.append(r)
        running = still
        lengths.append(step)
    active = sum(t[1] * t[4] for t in tasks)
    total = sum(lengths)
    return dict(steps=len(lengths), step_lengths=lengths, done_step=done, active=active, tasks=len(tasks),
                ideal_ratio=(active / (capacity * total)) if total > 0 else 0.0)


def event_schedule(counts, widths, ticks, capacity: int, batch: int):
    """The same rules with min_step = 0 as a discrete-event simulation: a heap
    of finish times; every distinct finish time is a step boundary, where the
    queue is scanned again.  Returns (finish time, boundary index) per sample."""
    tasks = tasks_of(counts, widths, ticks, batch)
    queue = list(range(len(tasks)))
    free = capacity
    heap = []                                  # (finish time, task)
    now = 0
    boundary = 0
    fin = np.zeros(int(sum(counts)), dtype=np.int64)
    idx = np.zeros(int(sum(counts)), dtype=np.int64)
    while True:
        waiting = []
        for q in queue:
            if tasks[q][1] <= free:
                free -= tasks[q][1]
                heapq.heappush(heap, (now + tasks[q][4], q))
            else:
                waiting.append(q)
        queue = waiting
        if not heap:
            break
        now = heap[0][0]
        while heap and heap[0][0] == now:
            _, q = heapq.heappop(heap)
            free += tasks[q][1]
            fin[tasks[q][2]:tasks[q][2] + tasks[q][3]] = now
            idx[tasks[q][2]:tasks[q][2] + tasks[q][3]] = boundary
        boundary += 1
    return fin, idx
