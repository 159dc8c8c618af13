"""Seeded synthetic inputs shared by the HIP path's tests/bench and the FP64 oracle.

This package only draws images and velocity fields. It holds none of the
registration method's arithmetic (no transport, no interpolation, no spectral
operators of the method): whatever input needs the method applied to it, such
as a reference image obtained by transporting a template, is composed by the
caller from these pieces.
"""

from .phantoms import (  # noqa: F401
    WORKLOADS,
    bandlimited_velocity,
    ellipsoid_phantom,
    gaussian_blobs,
    grid_coordinates,
    noise,
    trig_field,
)
