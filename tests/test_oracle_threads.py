"""The oracle's results do not depend on how many host threads run it: the
state and the FP64 mean velocity after several steps agree bit for bit with
one thread and with several (its only reduction, the mean velocity, sums in
a fixed order), so the CPU baseline may be timed on all host cores."""
import torch

import oracle as O
from lbm_inputs import percolating_x, random_mask


def test_oracle_bitwise_equal_across_thread_counts():
    m = percolating_x(random_mask((14, 12, 16), 0.3, 7))
    before = torch.get_num_threads()
    out = []
    try:
        for threads in (1, 3):
            torch.set_num_threads(threads)
            p = O.Problem(m, 0.9, 3 / 16, "E", (1e-5, 2e-6, -1e-6))
            fh = p.initial()
            for _ in range(12):
                fh, u = p.step(fh)
            out.append((fh.clone(), p.mean_velocity(u).clone()))
    finally:
        torch.set_num_threads(before)
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
