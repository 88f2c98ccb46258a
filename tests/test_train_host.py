"""Host logic of the training step: the Alg. 1 schedule and the position-rate decay."""
import math

import oracle
from paper_2506_06988_amd import train


def test_lambda_t_schedule_agrees_with_alg1_over_a_full_run():
    for i in range(0, 30001):
        assert train.lambda_t(i) == oracle.lambda_t_schedule(i)
    assert train.lambda_t(5000, lam=0.3, warmup=10, densify_until=20) == 0.0
    assert train.lambda_t(15, lam=0.3, warmup=10, densify_until=20) == 0.3


def test_position_rate_decay_is_log_linear():
    a, b, n = 1.6e-4, 1.6e-6, 30000
    assert math.isclose(train.exp_lr(0, a, b, n), a, rel_tol=1e-12)
    assert math.isclose(train.exp_lr(n, a, b, n), b, rel_tol=1e-12)
    assert math.isclose(train.exp_lr(n // 2, a, b, n), math.sqrt(a * b), rel_tol=1e-12)
    assert math.isclose(train.exp_lr(2 * n, a, b, n), b, rel_tol=1e-12)
