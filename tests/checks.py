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


def check_n_to_1_racing(values, statuses, nthreads=4, per=3, indices=None):
    """N-to-1 over a multiplex communicator with ANY_INDEX / ANY_TAG: every
    message arrives once, in order per sending thread, with a status naming
    its tag (10 * i + j) and, when given, its sender's stream index i."""
    assert sorted(values) == sorted(100 * i + j for i in range(nthreads) for j in range(per))
    for i in range(nthreads):
        mine = [v for v in values if v // 100 == i]
        assert mine == sorted(mine)
    for k, (v, st) in enumerate(zip(values, statuses)):
        assert st == (0, 10 * (v // 100) + v % 100, "SUCCESS", 4)
        if indices is not None:
            assert indices[k] == v // 100
