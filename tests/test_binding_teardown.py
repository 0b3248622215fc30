"""Teardown of the binding's native handles (host only).

Batch and Server handles still open at interpreter exit are closed by an
atexit hook while the HIP runtime and the library are alive; a handle's
__del__ does nothing once the interpreter is finalizing.
"""
import paper_1811_04165_amd as amber


class _Handle:
    def __init__(self):
        self.closed = 0

    def close(self):
        self.closed += 1
        amber._open_handles.discard(self)


def test_atexit_hook_closes_every_open_handle():
    hs = [_Handle() for _ in range(3)]
    for h in hs:
        amber._open_handles.add(h)
    amber._close_open_handles()
    assert [h.closed for h in hs] == [1, 1, 1]
    assert not any(h in amber._open_handles for h in hs)


def test_release_in_del_closes_when_not_finalizing():
    h = _Handle()
    amber._release_in_del(h)
    assert h.closed == 1


def test_release_in_del_swallows_errors():
    class Bad:
        def close(self):
            raise RuntimeError("closing failed")
    amber._release_in_del(Bad())   # no exception escapes a destructor
