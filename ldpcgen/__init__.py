"""Seeded synthetic inputs for NDGSBP decoding: LDPC parity-check matrices,
a GF(2) systematic encoder, BPSK/AWGN channel LLRs and the workload recipes.

This package holds none of the decoding method's arithmetic. It is the one
module that both the FP64 oracle (``oracle/``) and the HIP decoder
(``paper_1202_1060_amd``) consume, so that both see byte-identical inputs.

The paper's own codes (MacKay's (504,252) and (816,544) matrices, Sec. IV,
Figs. 2-3) are not available; seeded synthetic codes stand in for them.
"""
from .codes import Code, regular_code, qc_code, base_mask, QC_PROFILES, count_4cycles
from .gf2 import SystematicEncoder, gf2_rank
from .channel import ebn0_to_sigma, bpsk_awgn_llr, make_frames

__all__ = [
    "Code", "regular_code", "qc_code", "base_mask", "QC_PROFILES", "count_4cycles",
    "SystematicEncoder", "gf2_rank", "ebn0_to_sigma", "bpsk_awgn_llr", "make_frames",
]
