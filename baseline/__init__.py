"""CPU timing baselines for bench.py (not the oracle, not part of the GPU library)."""
