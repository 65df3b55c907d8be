"""Seeded synthetic inputs shared by the oracle's tests and the GPU path's
tests and benchmark: network weights (``weights``) and multi-view scenes
(``scenes``). Nothing here computes any step of the view-interpolation
network."""
