"""Seeded synthetic inputs for the network-aware container scheduler.

This module only draws random numbers and lays them out in the shared input
format (fat-tree capacities, background load, tenant requests, serving
traces).  It holds none of the scheduling method's arithmetic, so both the
FP64 oracle and the GPU library can be fed from it without sharing code.

Shared format (indices are the fat-tree conventions of the paper's DC graph,
section II-A, with the k-ary fat-tree of section IV-B):
  * hosts  h = p*(k/2)^2 + e*(k/2) + s        (pod p, edge switch e, slot s)
  * edge switch global index  eg = h // (k/2) = p*(k/2) + e
  * aggregation switch index  ag = p*(k/2) + a
  * core switch index         c  = a*(k/2) + j
  * link level 0 (host uplink)        index h
  * link level 1 (edge-aggregation)   index eg*(k/2) + a
  * link level 2 (aggregation-core)   index ag*(k/2) + j   (joins ag and core a*(k/2)+j)
  Every level has N = k^3/4 links.  Background load arrays are int32:
  host_used[2][N] (CPU cores, RAM GB) and link_used[3][N] (Mbps).
"""
from .gen import (FatTree, Instance, Request, make_instance, make_requests,
                  make_config, make_trace, CONFIGS, pack_requests, make_tiles, TILE_RANGES, make_event_workload)

__all__ = ["FatTree", "Instance", "Request", "make_instance", "make_requests",
           "make_config", "make_trace", "CONFIGS", "pack_requests", "make_tiles", "TILE_RANGES", "make_event_workload"]
