"""MI355X (gfx950) fast-HOG hot path: lookup-table bins, per-bin integral
images, four-corner cell histograms and linear window scores (arXiv:1703.06256).

Submodules:
    hog     -- Python binding of the C ABI in include/hog.h (libhog.so)
    inputs  -- seeded synthetic images and templates
    build   -- in-tree build of libhog.so with hipcc for gfx950
"""
