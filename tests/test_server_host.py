"""Server admission and argument checks that never reach the device (CPU
only): a stream whose declared budget does not fit is refused before
anything is allocated, and so are streams without a budget, bad server
arguments and calls on streams that were never admitted."""
import numpy as np
import pytest


def _cfg(budget):
    from paper_2608_06412_amd import default_config
    cfg = default_config(0.02, 0.06, max_blocks=1 << 12, max_points=1 << 14)
    cfg.hbm_budget = int(budget)
    return cfg


def test_admission_refused_by_budget():
    from paper_2608_06412_amd import AFError, Server
    from paper_2608_06412_amd.af import AF_EINVAL, AF_ENOMEM
    srv = Server(1 << 30, max_streams=2)
    with pytest.raises(AFError) as e:
        srv.admit(_cfg(2 << 30))
    assert e.value.code == AF_ENOMEM
    assert srv.reserved() == 0
    with pytest.raises(AFError) as e:
        srv.admit(_cfg(0))                       # no declared budget
    assert e.value.code == AF_EINVAL
    assert srv.step() == []                      # nothing admitted, nothing to run
    srv.close()


def test_bad_server_arguments_and_unknown_streams():
    from paper_2608_06412_amd import AFError, Server
    for budget, ns in ((0, 2), (1 << 30, 0), (1 << 30, 65)):
        with pytest.raises(AFError):
            Server(budget, max_streams=ns)
    srv = Server(1 << 30, max_streams=2)
    for call in (lambda: srv.prepare(0, [0, 0, 0], [1, 1, 1], 100, [0]),
                 lambda: srv.submit(1, np.zeros((3, 3), np.float32), [0, 0, 0], 0),
                 lambda: srv.release(0)):
        with pytest.raises(AFError):
            call()
    assert srv.pending(0) == -1
    srv.close()


def test_batch_threshold_arguments():
    from paper_2608_06412_amd import AFError, Server
    with pytest.raises(AFError):
        Server(1 << 30, max_streams=2, batch=-1)
    for b in (None, True, False, 1, 2, 8):
        Server(1 << 30, max_streams=2, batch=b).close()
