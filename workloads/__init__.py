"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds plain data only: problem descriptions (mesh, material,
scan path, solver options) and the seeded random draws that build them.  It
contains none of the method's arithmetic (no enthalpy, no element matrices,
no laser flux, no window rule), so both the CPU oracle and the GPU binding
can read it without sharing any computation.

The five workloads mirror the method's single-track / raster / served /
large-build cases on a laser powder-bed plate (Section 5 of the paper
describes the single-track and multi-track experiments this imitates).
"""
from .spec import (Mesh, Material, Track, ScanPath, Options, Workload,
                   FP64, MIXED, DN, COMPOSITE, ALTERNATE, CONSISTENT, SURFACE, VOLUME, default_material,
                   options_for)
from .configs import (single_track_1mm, single_track_2mm, raster_5mm,
                      served_tracks, raster_10mm,
                      single_track_3d, by_name, small_cases, k2_sweep_field)

__all__ = ["Mesh", "Material", "Track", "ScanPath", "Options", "Workload", "options_for",
           "FP64", "MIXED", "DN", "COMPOSITE", "ALTERNATE", "CONSISTENT", "SURFACE", "VOLUME",
           "default_material", "single_track_1mm", "single_track_2mm",
           "raster_5mm", "served_tracks", "raster_10mm", "single_track_3d", "by_name",
           "small_cases", "k2_sweep_field"]
