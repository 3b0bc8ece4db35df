"""CPU FP64 oracle (test infrastructure only).

Only `tests/`, the package smoke check and the benchmark's CPU-baseline leg may
import this package. The HIP library never calls it, and it shares no code with
the library.
"""
from .hloc_oracle import (FLAG_EMPTY, FLAG_LOW_CONFIDENCE, TIE_REL, aggregate, fft_magnitude,
                          localize, localize_labels, region_means, retrieve, search_rows, select_regions, sq_dist,
                          tile_of)

__all__ = ["FLAG_EMPTY", "FLAG_LOW_CONFIDENCE", "TIE_REL", "aggregate", "fft_magnitude",
           "localize", "localize_labels", "region_means", "retrieve", "search_rows", "select_regions", "sq_dist",
           "tile_of"]
