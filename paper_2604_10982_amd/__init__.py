"""MI355X-native rasterizer for Psi-Map panoptic surfel maps (arXiv 2604.10982).

The HIP library is loaded lazily on first use (``paper_2604_10982_amd.psm``);
importing the package, or its ``scenes`` module, touches no GPU.
"""
__all__ = ["scenes"]
