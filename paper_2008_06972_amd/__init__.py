"""MI355X (gfx950) spatio-temporal LiDAR range-image encoder.

The encoder of Feng, Liu and Zhu, "Real-Time Spatio-Temporal LiDAR Point
Cloud Compression", as hand-written HIP kernels behind the C ABI of
``include/pc.h``; :mod:`paper_2008_06972_amd.pcc` is the ctypes binding and
:mod:`paper_2008_06972_amd.synth` the seeded scene generator used for inputs.
"""
__version__ = "1.0"
