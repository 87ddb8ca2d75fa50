"""Checks shared by the oracle tests and the GPU tests (no method arithmetic)."""


def check_competing(values, statuses, nsend=3, per=4):
    """Every message arrives exactly once, per-sender order holds, statuses
    agree with the payloads."""
    assert sorted(values) == sorted(1000 * q + i for q in range(1, nsend + 1) for i in range(per))
    for q in range(1, nsend + 1):
        mine = [v for v in values if v // 1000 == q]
        assert mine == sorted(mine)
    for v, st in zip(values, statuses):
        assert st == (v // 1000, 7 + v % 1000, "SUCCESS", 4)
