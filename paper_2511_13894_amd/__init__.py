"""MI355X-native restarted PDHG with the corner-push phase of arXiv 2511.13894."""
