"""FP64 CPU oracle of the LB-IMB-DEM step (test infrastructure only)."""
