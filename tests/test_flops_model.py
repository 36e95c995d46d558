"""The algorithmic work model behind the roofline figures: its closed forms
for a closed polygon and a free segment, and its per-instance sum."""
import numpy as np

from paper_2607_04310_amd import flops, inputs


def test_closed_forms():
    for m in range(3, 17):
        for mi in range(3, 17):
            assert flops.flops_pair(m, mi, mi) == 32 * m * mi + 3 * mi * mi + 22 * mi + 5 * m + 1
        assert flops.flops_pair(m, 1, 2) == 37 + 53 * m
    assert flops.flops_pair(6, 4, 4) == 935 and flops.flops_pair(4, 4, 4) == 669


def test_instance_sum_and_shapes():
    inst = inputs.c2(0)
    assert flops.flops_instance(6, inst.N, inst.edges, inst.obst_off) == 50 * 4096 * 935
    # a free segment and an open chain of three edges (six V_obs points)
    edges = np.array([[0, 0, 1, 0], [2, 0, 3, 0], [3, 0, 3, 1], [3, 1, 2, 2]], np.float32)
    shapes = flops.obstacle_shapes(edges, np.array([0, 1, 4]))
    assert shapes == [(1, 2), (3, 6)]
    assert flops.flops_instance(4, 2, edges, [0, 1, 4]) == 2 * (flops.flops_pair(4, 1, 2)
                                                                + flops.flops_pair(4, 3, 6))
