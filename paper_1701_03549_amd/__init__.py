"""MI355X-native stochastic CA fire simulation and fitting (Denham & Laneri, arXiv 1701.03549)."""
