"""Seeded synthetic inputs (OFDM grids, weight blobs, request mixes) for CoNet-Rx.

Nothing here computes the receiver network; it only generates what the network reads.
"""
from .ofdm import SimConfig, simulate_slot, simulate_batch, features_fast, pilot_mask, data_mask, qam_map
from .weights import ModelConfig, blob_layout, blob_size, make_blob, split_blob
from .workloads import WORKLOADS, workload
