"""Seeded synthetic inputs (rigid water boxes and gas-phase clusters).

This package only draws random numbers and lays out arrays; it holds none of
the method's arithmetic (no fields, no energies, no solver).  Both the CPU
oracle's tests and the GPU path's tests/bench draw their inputs from here.
"""
from .water import (CONFIGS, water_box, water_box_ortho, water_cluster, config_system,
                    water_frames, water_md, water_lone_pairs, water_ct, WATER_SITES,
                    CT_SITES, SITE_NAMES)

__all__ = ["CONFIGS", "water_box", "water_box_ortho", "water_cluster", "config_system",
           "water_frames", "water_md", "water_lone_pairs", "water_ct", "WATER_SITES",
           "CT_SITES", "SITE_NAMES"]
