"""pdfx: batched parton-density and alpha_s interpolation on AMD MI355X (gfx950)."""
