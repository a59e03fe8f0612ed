"""Hand-made k = 4 data centers and a request for the selection pins:
server 8 scores highest for the last container and passes every per-peer
check, but its joint commit fails, so the next server must take it."""
import numpy as np

from workloads import Request, make_instance

N4 = 16   # servers of a k = 4 fat-tree


def empty():
    return make_instance(4, 32, 256, 10000, 10000, 10000)


def loaded():
    """k = 4, 1,000 Mbps links.  Residual CPU: servers 0 and 4 have 32
    cores, server 8 30, server 12 29, every other server 10.  Server 8's
    edge switch (switch 4) has 500 Mbps left towards aggregation switch 0
    and 100 towards aggregation switch 1; every other link is free."""
    inst = make_instance(4, 32, 256, 1000, 1000, 1000)
    cpu = np.full(N4, 10, np.int32)
    cpu[[0, 4]] = 32
    cpu[8] = 30
    cpu[12] = 29
    hu = np.zeros((2, N4), np.int32)
    hu[0] = 32 - cpu
    lu = np.zeros((3, N4), np.int32)
    lu[1, 4 * 2 + 0] = 500
    lu[1, 4 * 2 + 1] = 900
    inst.host_used, inst.link_used = hu, lu
    return inst


# Containers 0 and 1 need 20 cores, container 2 one core and 300 Mbps to
# each of them; one GB of RAM each.
REQ = Request(np.array([20, 20, 1], np.int32), np.array([1, 1, 1], np.int32),
              np.array([[0, 2, 300], [1, 2, 300]], np.int32))


def split_fits():
    """loaded() with 600 and 0 Mbps left on edge switch 4's uplinks: the
    same per-peer checks, but both paths fit through the first uplink."""
    inst = loaded()
    inst.link_used[1, 8], inst.link_used[1, 9] = 400, 1000
    return inst


def peer_cut(uplink0=500):
    """k = 4, 1,000 Mbps links.  Residual CPU: server 0 has 32 cores,
    server 1 14, every other server 10; server 0's uplink has uplink0 Mbps
    left, every other link is free."""
    inst = make_instance(4, 32, 256, 1000, 1000, 1000)
    cpu = np.full(N4, 10, np.int32)
    cpu[0], cpu[1] = 32, 14
    hu = np.zeros((2, N4), np.int32)
    hu[0] = 32 - cpu
    lu = np.zeros((3, N4), np.int32)
    lu[0, 0] = 1000 - uplink0
    inst.host_used, inst.link_used = hu, lu
    return inst


# Containers 0 and 1 need 12 cores (both go to server 0, leaving it 8),
# container 2 one core and 300 Mbps to each of them.
REQ_CUT = Request(np.array([12, 12, 1], np.int32), np.array([1, 1, 1], np.int32),
                  np.array([[0, 2, 300], [1, 2, 300]], np.int32))
