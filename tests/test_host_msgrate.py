"""Host message-rate model (CPU only): every policy delivers every message
once and in order, checked against the closed form of its checksum, and bad
arguments are refused."""
import pytest

from paper_2208_13707_amd import driver as D

MASK = (1 << 64) - 1


def closed_form(npairs, n):
    # sum over pairs i and messages k < n of (i * 2^40 + k) * (k + 1):
    # sum k (k + 1) = (n - 1) n (n + 1) / 3 and sum (k + 1) = n (n + 1) / 2
    s = 0
    for i in range(npairs):
        s += (i << 40) * (n * (n + 1) // 2) + (n - 1) * n * (n + 1) // 3
    return s & MASK


def brute(npairs, n):
    return sum((i * 2**40 + k) * (k + 1) for i in range(npairs) for k in range(n)) & MASK


def test_closed_form_against_brute_force():
    for p, n in ((1, 1), (2, 7), (3, 130)):
        assert closed_form(p, n) == brute(p, n)


@pytest.mark.parametrize("policy", ["global", "per_context", "stream"])
@pytest.mark.parametrize("npairs,msgs,window", [(1, 1, 1), (1, 1000, 1), (3, 10007, 64),
                                                 (2, 5000, 1024), (4, 2049, 1000)])
def test_every_message_once_in_order(policy, npairs, msgs, window):
    rc, rate, ck = D.mpixs_drv_host_msgrate(npairs, policy, msgs, window)
    assert rc == 0 and rate > 0
    assert ck == closed_form(npairs, msgs)


@pytest.mark.parametrize("args", [(0, 0, 10, 8), (257, 0, 10, 8), (1, 3, 10, 8), (1, -1, 10, 8),
                                  (1, 0, 0, 8), (1, 0, 10, 0), (1, 0, 10, 1025)])
def test_bad_arguments(args):
    rc, _, _ = D.mpixs_drv_host_msgrate(*args)
    assert rc == 1
