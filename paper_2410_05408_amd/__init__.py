"""MI355X-native oblate-planet transit light curves (arXiv:2410.05408)."""
