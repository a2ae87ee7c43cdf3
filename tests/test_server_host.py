"""Serving loop, host side (no GPU): argument checking and the state of an empty server.
The scheduler thread and device memory start with the first tenant, so none of this
touches a GPU."""
import ctypes as C

import pytest

import paper_2511_00737_amd as ep


def _create(budget=1 << 30, streams=2, max_batch=0):
    h = C.c_void_p()
    st = ep.lib().ephdc_server_create(budget, streams, max_batch, C.byref(h))
    return st, h


def test_rejects_bad_configuration():
    assert _create(budget=1 << 20)[0] == ep.ERR_ARG  # below 64 MiB
    assert _create(streams=0)[0] == ep.ERR_ARG
    assert _create(streams=9)[0] == ep.ERR_ARG
    assert b"streams" in ep.lib().ephdc_last_error()


def test_empty_server_errors_and_stats():
    st, h = _create()
    assert st == ep.OK
    try:
        tk = C.c_uint64()
        fake = C.c_void_p(0x10000)  # never dereferenced: the tenant check fails first
        assert ep.lib().ephdc_server_submit(h, 0, fake, 10, fake, None, C.byref(tk)) == ep.ERR_ARG
        assert b"unknown tenant" in ep.lib().ephdc_last_error()
        assert ep.lib().ephdc_server_submit(h, 0, None, 10, fake, None, C.byref(tk)) == ep.ERR_ARG
        state = C.c_int32()
        assert ep.lib().ephdc_server_query(h, 12345, C.byref(state), None) == ep.ERR_ARG
        assert ep.lib().ephdc_server_wait(h, 0, 1.0) == ep.OK  # nothing waits or runs
        assert ep.lib().ephdc_server_wait(h, 7, 1.0) == ep.ERR_ARG  # unknown ticket
        assert ep.lib().ephdc_server_release(h, 7) == ep.ERR_ARG  # unknown ticket
        out = (C.c_double * 14)()
        assert ep.lib().ephdc_server_stats(h, out) == ep.OK
        stats = dict(zip(ep.Server.STATS, out))
        assert stats["submitted"] == 0 and stats["completed"] == 0 and stats["batches"] == 0
        assert stats["failed"] == 0 and stats["tickets"] == 0
        assert stats["budget_bytes"] == 1 << 30
    finally:
        assert ep.lib().ephdc_server_destroy(h) == ep.OK


def test_python_wrapper_rejects_unknown_tenant():
    sv = ep.Server(1 << 30)
    try:
        with pytest.raises(ep.EphdcError):
            sv.submit(3, None, 1, None)
    finally:
        sv.close()
