"""MI355X-native SAP-preconditioned FGCR solver for the Wilson-clover Dirac
equation (the method of Heybrock et al., SC14, arXiv:1412.2629)."""
