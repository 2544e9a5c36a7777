"""Two-layer shallow-water AMR hot path on MI355X (see the C-ABI header in include/)."""
