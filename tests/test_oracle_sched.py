"""Pins of the round scheduler oracle (finest-first greedy, eq. batch reading)
on cases worked out by hand."""
import math

from oracle import sched


def test_batch_sizes_fall_with_the_unassigned_samples():
    # 100 samples on 4 lanes, capacity 40, device fill 5: per = 25, maximum
    # ceil(25 * 0.618) = 16, minimum max(ceil(0.25), min(40, 5)) = 5; each batch
    # ceil(left / 4) clamped:
    #   left 100 -> 25 -> 16;  84 -> 21 -> 16;  68 -> 17 -> 16;  52 -> 13;  39 -> 10;
    #   29 -> 8;  21 -> 6;  15 -> 4 -> 5;  10 -> 3 -> 5;  5 -> 2 -> 5
    assert sched.batch_sizes(100, 4, 40, 5) == [16, 16, 16, 13, 10, 8, 6, 5, 5, 5]


def test_batch_sizes_floor_and_one_lane():
    # the device-filling floor keeps a small level in one batch
    assert sched.batch_sizes(100, 4, 1000, 125) == [100]
    # ... and never exceeds the capacity: a 256^3 batch of 16 (fill 32) stays whole
    assert sched.batch_sizes(16, 4, 16, 32) == [16]
    # one lane: capacity-sized batches
    assert sched.batch_sizes(2500, 1, 1024, 512) == [1024, 1024, 452]
    assert sched.batch_sizes(0, 4, 10, 1) == []


def test_maximum_is_the_golden_fraction():
    # the first batch of a level is phi^-1 of its per-lane share
    per = 1000
    assert sched.batch_sizes(4 * per, 4, 10 ** 6, 125000) == [4000]   # the floor takes all that is left
    b = sched.batch_sizes(4 * per, 4, 8000, 1000)[0]                  # floor 1000, maximum 619
    assert b == 1000
    b = sched.batch_sizes(4 * per, 4, 800, 100)[0]                    # floor 100, maximum ceil(618.03) = 619
    assert b == 619 and abs(b / per - 0.618) < 2e-3


def test_level_cap_follows_the_dof_budget():
    # 5 levels from 8^3: the 128^3 pair has 2048383 + 250047 unknowns, the 8^3
    # level 343; 1024 samples on the finest mesh -> min(1024 * 6700.4, 65536)
    assert sched.level_cap(8, 5, 4, 1024) == 1024
    assert sched.level_cap(8, 5, 0, 1024) == 65536
    # 64^3 / 32^3 pair over the 32^3 / 16^3 pair: 279838 / 33166 = 8.437...
    assert sched.level_cap(16, 3, 1, 4) == math.floor(4 * 279838 / 33166)


def test_greedy_assignment_by_hand():
    # meshes 4, 8, 16 (levels 0..2), requests 5, 3, 2 samples, 2 lanes, capacity 2, fill 1
    # batches: level 2 [1, 1]; level 1 [2, 1]; level 0 [2, 2, 1]
    # tasks by decreasing mesh with their work (samples x interior unknowns):
    #   16^3: L2 fine 3375, L2 fine 3375
    #   8^3:  L2 coarse 343, L2 coarse 343, L1 fine 686, L1 fine 343
    #   4^3:  L1 coarse 54, L1 coarse 27, L0 54, L0 54, L0 27
    # least-loaded lane each time (loads after each step):
    #   (3375,0) (3375,3375) (3718,3375) (3718,3718) (4404,3718) (4404,4061)
    #   (4404,4115) (4404,4142) (4404,4196) (4404,4250) (4404,4277)
    t = sched.plan(4, [(0, 0, 5), (1, 0, 3), (2, 0, 2)], 2, [2, 2, 2], [1, 1, 1])
    assert [x["lane"] for x in t] == [0, 1, 0, 1, 0, 1, 1, 1, 1, 1, 1]
    assert [(p["level"], x["n"], p["first"], p["count"]) for x in t for p in x["parts"]] == [
        (2, 16, 0, 1), (2, 16, 1, 1),
        (2, 8, 0, 1), (2, 8, 1, 1), (1, 8, 0, 2), (1, 8, 2, 1),
        (1, 4, 0, 2), (1, 4, 2, 1), (0, 4, 0, 2), (0, 4, 2, 2), (0, 4, 4, 1)]


def test_packing_pairs_levels_on_one_mesh_by_hand():
    # the same round with packing, capacities 2 / 3 / 2 for levels 0 / 1 / 2:
    # level 1 batches (3 samples, cap 3, fill 1): per 2, most ceil(1.24) = 2 -> [2, 1]
    # 8^3 (mesh level 1, cap 3): coarse L2 [1, 1] with fine L1 [2, 1] -> pairs
    #   (1 + 2 = 3 fits) and (1 + 1 = 2 fits): two tasks of 3 and 2 samples
    # 4^3 (mesh level 0, cap 2): coarse L1 [2, 1] with fine L0 [2, 2, 1] ->
    #   2 + 2 = 4 > 2: apart; 1 + 2 = 3 > 2: apart; then fine L0 [1] alone
    # work: 16^3 3375, 3375; 8^3 1029, 686; 4^3 54, 54, 27, 54, 27
    # lanes: (3375,0) (3375,3375) (4404,3375) (4404,4061) (4404,4115) (4404,4169)
    #        (4404,4196) (4404,4250) (4404,4277)
    t = sched.plan(4, [(0, 0, 5), (1, 0, 3), (2, 0, 2)], 2, [2, 3, 2], [1, 1, 1], pack=True)
    assert [[(p["level"], p["first"], p["count"]) for p in x["parts"]] for x in t] == [
        [(2, 0, 1)], [(2, 1, 1)],
        [(2, 0, 1), (1, 0, 2)], [(2, 1, 1), (1, 2, 1)],
        [(1, 0, 2)], [(0, 0, 2)], [(1, 2, 1)], [(0, 2, 2)], [(0, 4, 1)]]
    assert [x["n"] for x in t] == [16, 16, 8, 8, 4, 4, 4, 4, 4]
    assert [x["lane"] for x in t] == [0, 1, 0, 1, 1, 1, 1, 1, 1]


def test_one_lane_keeps_request_order_by_mesh():
    t = sched.plan(8, [(1, 32, 4), (0, 32, 4)], 1, [64, 64], [8, 8])
    assert [(p["level"], x["n"], x["lane"]) for x in t for p in x["parts"]] == [(1, 16, 0), (1, 8, 0), (0, 8, 0)]
    # with packing the two 8^3 solves share one task
    t = sched.plan(8, [(1, 32, 4), (0, 32, 4)], 1, [64, 64], [8, 8], pack=True)
    assert [[p["level"] for p in x["parts"]] for x in t] == [[1], [1, 0]]
