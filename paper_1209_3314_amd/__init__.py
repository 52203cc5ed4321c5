"""MI355X-native irregular wavefront propagation (IWPP), arXiv 1209.3314."""
