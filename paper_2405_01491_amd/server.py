"""Python handle of the continuous-batching server (nnp_server_* / nnp_submit /
nnp_poll in include/nnp.h).  Marshalling only: admission, batching, launches
and completion tracking run in libnnp's native scheduler thread."""
import ctypes

import numpy as np

from . import _lib
from ._lib import NNPError, check, lib


class Server:
    def __init__(self, model, arena_bytes=64 << 20, max_slots=4096, max_inflight=4):
        self.model = model
        h = ctypes.c_void_p()
        check(lib().nnp_server_create(model.handle, int(arena_bytes), int(max_slots), int(max_inflight),
                                      ctypes.byref(h)), "nnp_server_create")
        self.handle = h
        self.n_atoms = {}

    def close(self):
        if getattr(self, "handle", None):
            lib().nnp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        c, l, b = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().nnp_server_stats(self.handle, ctypes.byref(c), ctypes.byref(l), ctypes.byref(b)),
              "nnp_server_stats")
        return {"completed": c.value, "launches": l.value, "batched_requests": b.value}


def nnp_submit(server, species, pos):
    """Submit one structure (host arrays).  Returns the ticket, or None if the
    server is full right now (NNP_E_BUSY); raises NNPError otherwise."""
    sp = np.ascontiguousarray(np.asarray(species, dtype=np.int32))
    x = np.ascontiguousarray(np.asarray(pos, dtype=np.float32))
    t = ctypes.c_uint64()
    st = lib().nnp_submit(server.handle, len(sp), sp.ctypes.data_as(ctypes.c_void_p),
                          x.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t))
    if st == _lib.NNP_E_BUSY:
        return None
    check(st, "nnp_submit")
    server.n_atoms[t.value] = len(sp)
    return t.value


def nnp_poll(server, ticket):
    """None while pending; (energy float, forces [n,3] float32) once done."""
    n = server.n_atoms[ticket]
    e = ctypes.c_double()
    F = np.empty((n, 3), dtype=np.float32)
    st = lib().nnp_poll(server.handle, ctypes.c_uint64(ticket), ctypes.byref(e), F.ctypes.data_as(ctypes.c_void_p))
    if st == _lib.NNP_E_PENDING:
        return None
    del server.n_atoms[ticket]
    check(st, "nnp_poll")
    return e.value, F
