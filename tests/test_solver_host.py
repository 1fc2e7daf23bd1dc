"""Host logic of the differentiable rollout (CPU only): the checkpoint
interval picked from the free device memory."""
import torch

from paper_0903_4044_amd import solver


def test_auto_every_keeps_every_state_when_the_trajectory_fits():
    f0 = torch.zeros(1000, dtype=torch.float32)  # 4000 B per state
    # 201 states (200 steps + the final one) in half of the free memory
    assert solver.auto_every(f0, 200, free_bytes=2 * 201 * 4000) == 1
    assert solver.auto_every(f0, 200, free_bytes=2 * 201 * 4000 - 1) > 1


def test_auto_every_smallest_interval_that_fits():
    f0 = torch.zeros(1000, dtype=torch.float64)  # 8000 B per state
    # budget of 30 states: ceil(200/e) + e <= 30 first holds at e = 10 (20 + 10)
    assert solver.auto_every(f0, 200, free_bytes=2 * 30 * 8000) == 10
    assert solver.auto_every(f0, 200, free_bytes=2 * 29 * 8000) > 10


def test_auto_every_falls_back_to_square_root():
    f0 = torch.zeros(10, dtype=torch.float32)
    assert solver.auto_every(f0, 200, free_bytes=1) == 15  # ceil(sqrt(200))
    assert solver.auto_every(f0, 1, free_bytes=1) == 1


def test_auto_mode_takes_records_when_states_and_records_fit():
    f0 = torch.zeros(1000, dtype=torch.float32)  # 4000 B per state
    rec = 5000  # bytes per step record
    need = 201 * 4000 + 200 * rec  # states f^0 .. f^200 and 200 records
    assert solver.auto_mode(f0, 200, rec, fraction=0.6, free_bytes=int(need / 0.6) + 1) == "record"
    assert solver.auto_mode(f0, 200, rec, fraction=0.6, free_bytes=int(need / 0.6) - 10) == "checkpoint"
