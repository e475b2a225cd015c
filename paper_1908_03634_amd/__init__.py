"""MI355X-native MAC-projection solve (MAESTROeX low Mach number method).

The GPU library is loaded lazily on first use, so that the input generators in
`workloads` import without it.  Nothing here falls back to a CPU path: every
solve runs through the HIP library and fails loudly when it is missing.
"""
__all__ = ["workloads"]
