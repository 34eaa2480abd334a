"""MI355X-native one-step solver for spherical quasi-geostrophic convection
(Chebyshev-integration / tau radial scheme, Fourier in azimuth, IMEX time
stepping), after Gastine, arXiv:1902.07092."""
